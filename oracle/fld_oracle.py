"""FP64 CPU oracle for one implicit FLD radiation-energy step.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
reference the GPU library is checked against.  Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the library
itself never does, and the two share no code (only the seeded input
generators in ``fld_workloads`` serve both).

What it computes (Chen et al., "Guangqi", Section 3.2.1):

* Flux-limited diffusion closure F = -D grad E, D = c lambda(R) / (kappa_R rho)
  (Section 2, eqs. for the FLD flux and the reduced gradient R).
* Backward-Euler discretisation of the radiation-energy equation coupled to
  the gas energy, with the T^4 term linearised to first order about T^n
  (Section 3.2.1, linear system and Taylor expansion of T^4).
* Face coefficients: interface opacity interpolated from the two cell centres,
  interface E the average of the two neighbours, D from the limiter
  (Section 3.2.1, interface diffusion coefficient).
* Matrix elements phi_1..phi_11 and psi_5, psi_6, psi_11 with
  beta = kappa rho c dt, alpha = dt / (distance of volume centres), g = dS/dV
  (Section 3.2.1, coefficient list and the alpha definition).

Because psi rows couple only E_ij and T_ij, T is eliminated exactly
(T = (psi_11 - psi_5 E)/psi_6) and the remaining E system, multiplied by the
cell volume, is symmetric positive definite:

    M_ii = dV (1 + beta f) + sum_faces W,   M_i,nb = -W,
    rhs_i = dV (E^n + beta f a_R T^4),      f = C_V / (C_V + 4 beta a_R T^3),
    W = dt dS D / h.

The oracle solves that system with a sparse direct factorisation (SciPy's
SuperLU), then recovers T^{n+1} from the psi row.  Readings of points the
paper leaves open (all listed in the design notes):

* D is positive (the minus sign in the printed interface coefficient
  contradicts F = -D grad E and phi_5 = 1 - phi_1 - ...).
* The exchange sign follows the conservation laws of Section 2 and the
  phi/psi list (not the sign written in the time-discrete pair).
* kappa_e = kappa_P (Section 2, emissivity paragraph); S_g = 0; S_adv = 0
  unless face mass fluxes are given (``advection_volume_term``).
* C_V is per unit volume; inputs give c_v per gram, so C_V = rho c_v.
* Interface sigma = kappa_R rho is the distance-weighted mean of the two
  cells (harmonic mean of the diffusivities); interface E is the linear
  interpolation to the face (equal weights on a uniform grid).
* R uses the face-normal two-point difference.
* The default limiter is Levermore-Pomraning, lambda = (coth R - 1/R)/R; the
  paper's Minerbo form and the pure-diffusion value 1/3 are options.
* Boundary faces: reflecting and axis faces carry no flux; Dirichlet face,
  Dirichlet ghost, fixed inward flux and free-streaming outflow as documented
  in ``boundary_terms``.

Parity status: every function here is pinned by tests/test_oracle_*.py
against closed forms, invariants, the paper's worked numbers, a dense solve
of the paper's coupled (E, T) system and brute force; none is "parity
unpinned".
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# cgs constants (the paper prints none of them)
C_LIGHT = 2.99792458e10          # cm s^-1
SIGMA_SB = 5.670374419e-5        # erg cm^-2 s^-1 K^-4
A_RAD = 4.0 * SIGMA_SB / C_LIGHT  # radiation constant a_R, erg cm^-3 K^-4

CARTESIAN, SPHERICAL = 0, 1
REFLECT, DIRICHLET_FACE, DIRICHLET_GHOST, FLUX_IN, FREE_STREAM, AXIS, MILNE = range(7)
LIMITER_LP, LIMITER_MINERBO, LIMITER_DIFFUSION = range(3)


# ---------------------------------------------------------------------------
# flux limiters (Section 2: FLD closure, asymptotic limits, limiter forms)
# ---------------------------------------------------------------------------

def limiter_lp(R):
    """Levermore-Pomraning limiter lambda(R) = (coth R - 1/R) / R.

    For R < 0.1 the Taylor series 1/3 - R^2/45 + 2R^4/945 - R^6/4725
    + 2R^8/93555 is used: the closed form cancels catastrophically there.
    """
    R = np.asarray(R, dtype=np.float64)
    out = np.empty_like(R)
    small = R < 0.1
    Rs = R[small]
    R2 = Rs * Rs
    out[small] = 1.0 / 3.0 + R2 * (-1.0 / 45.0 + R2 * (2.0 / 945.0 + R2 * (-1.0 / 4725.0 + R2 * (2.0 / 93555.0))))
    Rl = R[~small]
    out[~small] = (1.0 / np.tanh(Rl) - 1.0 / Rl) / Rl
    return out


def limiter_minerbo(R):
    """Minerbo-type limiter printed in Section 2 (piecewise at R = 3/2)."""
    R = np.asarray(R, dtype=np.float64)
    lo = 2.0 / (3.0 + np.sqrt(9.0 + 12.0 * R * R))
    hi = 1.0 / (1.0 + R + np.sqrt(1.0 + 2.0 * R))
    return np.where(R <= 1.5, lo, hi)


def limiter_diffusion(R):
    """lambda = 1/3: the optically thick (pure diffusion) limit."""
    return np.full_like(np.asarray(R, dtype=np.float64), 1.0 / 3.0)


LIMITERS = {LIMITER_LP: limiter_lp, LIMITER_MINERBO: limiter_minerbo, LIMITER_DIFFUSION: limiter_diffusion}


# ---------------------------------------------------------------------------
# grid metrics (Section 3.2.1: g = dS/dV, alpha from volume centres)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Metrics:
    nx: int
    ny: int
    dV: np.ndarray     # [ny, nx]
    dSx: np.ndarray    # [ny, nx+1]  area of x/r faces (face i is left of cell i)
    dSy: np.ndarray    # [ny+1, nx]  area of y/theta faces
    hLx: np.ndarray    # [ny, nx+1]  distance from the centre of cell i-1 to face i (0 at i=0)
    hRx: np.ndarray    # [ny, nx+1]  distance from face i to the centre of cell i (0 at i=nx)
    hLy: np.ndarray    # [ny+1, nx]
    hRy: np.ndarray    # [ny+1, nx]


def theta_centre_offset(a, h):
    """th_c - a for the cell [a, a + h] of a spherical-polar grid.

    th_c is the volume-weighted mean angle (weight sin th), i.e.
    th_c - a = int_0^h u sin(a + u) du / int_0^h sin(a + u) du
             = (sin a S1 + cos a S2) / (sin a sin h + cos a C1),
    S1 = int u cos u = h sin h - C1, S2 = int u sin u = sin h - h cos h,
    C1 = 1 - cos h = 2 sin^2(h/2).  S2 uses its Taylor series
    h^3/3 - h^5/30 + h^7/840 - h^9/45360 + h^11/3991680 - h^13/518918400
    for h < 0.3 (the closed form cancels there).
    """
    a = np.asarray(a, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    C1 = 2.0 * np.sin(0.5 * h) ** 2
    S1 = h * np.sin(h) - C1
    h2 = h * h
    series = h * h2 * (1.0 / 3.0 + h2 * (-1.0 / 30.0 + h2 * (1.0 / 840.0 + h2 * (-1.0 / 45360.0 + h2 * (
        1.0 / 3991680.0 + h2 * (-1.0 / 518918400.0))))))
    S2 = np.where(h < 0.3, series, np.sin(h) - h * np.cos(h))
    return (np.sin(a) * S1 + np.cos(a) * S2) / (np.sin(a) * np.sin(h) + np.cos(a) * C1)


def metrics(geom: int, xf: np.ndarray, yf: np.ndarray) -> Metrics:
    """Cell volumes, face areas and centre-to-face distances.

    Cartesian (x, y): dV = dx dy, dS_x = dy, dS_y = dx, centres at midpoints.
    Spherical-polar (r, theta), the azimuthal 2 pi dropped throughout:
      dV = (r+^3 - r-^3)/3 (cos th- - cos th+),
      dS_r = r_f^2 (cos th- - cos th+),  dS_th = sin th_f (r+^2 - r-^2)/2,
      volume centres r_c = 3/4 (r+^4 - r-^4)/(r+^3 - r-^3) and
      th_c = (sin th+ - sin th- - th+ cos th+ + th- cos th-)/(cos th- - cos th+);
      distances along theta are arc lengths at r_c.
    The spherical forms are evaluated in algebraically identical,
    cancellation-free arrangements (see theta_centre_offset).
    """
    xf = np.asarray(xf, dtype=np.float64)
    yf = np.asarray(yf, dtype=np.float64)
    nx, ny = xf.size - 1, yf.size - 1
    xm, xp = xf[:-1], xf[1:]
    ym, yp = yf[:-1], yf[1:]
    if geom == CARTESIAN:
        xc = 0.5 * (xm + xp)
        yc = 0.5 * (ym + yp)
        Vx, Vy = xp - xm, yp - ym
        dV = Vy[:, None] * Vx[None, :]
        dSx = np.broadcast_to(Vy[:, None], (ny, nx + 1)).copy()
        dSy = np.broadcast_to(Vx[None, :], (ny + 1, nx)).copy()
        arc = np.ones(nx)
    elif geom == SPHERICAL:
        # same closed forms, evaluated without cancellation for thin cells:
        # r+^3 - r-^3 and r+^4 - r-^4 factorised, cos th- - cos th+ as a product
        # of sines, and the theta centre as an offset from the lower face.
        dr = xp - xm
        q = xp * xp + xp * xm + xm * xm
        Vx = dr * q / 3.0
        xc = 0.75 * (xp + xm) * (xp * xp + xm * xm) / q
        off_r = dr * (6.0 * xm * xm + 8.0 * xm * dr + 3.0 * dr * dr) / (4.0 * q)  # r_c - r-
        dth = yp - ym
        Vy = 2.0 * np.sin(0.5 * (ym + yp)) * np.sin(0.5 * dth)
        off_t = theta_centre_offset(ym, dth)  # th_c - th-
        dV = Vy[:, None] * Vx[None, :]
        dSx = Vy[:, None] * (xf ** 2)[None, :]
        dSy = np.sin(yf)[:, None] * (0.5 * dr * (xp + xm))[None, :]
        hLx = np.zeros((ny, nx + 1))
        hRx = np.zeros((ny, nx + 1))
        hLx[:, 1:] = (dr - off_r)[None, :]
        hRx[:, :-1] = off_r[None, :]
        hLy = np.zeros((ny + 1, nx))
        hRy = np.zeros((ny + 1, nx))
        hLy[1:, :] = (dth - off_t)[:, None] * xc[None, :]
        hRy[:-1, :] = off_t[:, None] * xc[None, :]
        return Metrics(nx, ny, dV, dSx, dSy, hLx, hRx, hLy, hRy)
    else:
        raise ValueError("unknown geometry")
    hLx = np.zeros((ny, nx + 1))
    hRx = np.zeros((ny, nx + 1))
    hLx[:, 1:] = (xf[1:] - xc)[None, :]
    hRx[:, :-1] = (xc - xf[:-1])[None, :]
    hLy = np.zeros((ny + 1, nx))
    hRy = np.zeros((ny + 1, nx))
    hLy[1:, :] = (yf[1:] - yc)[:, None] * arc[None, :]
    hRy[:-1, :] = (yc - yf[:-1])[:, None] * arc[None, :]
    return Metrics(nx, ny, dV, dSx, dSy, hLx, hRx, hLy, hRy)


# ---------------------------------------------------------------------------
# assembly
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class BCSpec:
    kind: int = REFLECT
    value: float = 0.0                   # Dirichlet face: T_b [K]; flux-in: F_in
    ghost: Optional[np.ndarray] = None   # Dirichlet ghost: ghost-cell E along the side


@dataclasses.dataclass
class Assembled:
    met: Metrics
    W_x: np.ndarray     # [ny, nx+1] conductance dt dS D / h of x faces (boundary columns: boundary faces)
    W_y: np.ndarray     # [ny+1, nx]
    D_x: np.ndarray     # [ny, nx+1] diffusion coefficient of x faces (0 where no flux)
    D_y: np.ndarray
    diag: np.ndarray    # [ny, nx]
    rhs: np.ndarray     # [ny, nx]
    CV: np.ndarray
    beta: np.ndarray
    X: np.ndarray       # 4 beta a_R T^3
    f: np.ndarray       # C_V / (C_V + X)
    bdiag: np.ndarray   # boundary contribution to the diagonal
    brhs: np.ndarray    # boundary contribution to the right-hand side
    M: sp.csr_matrix


def face_D(sigL, sigR, hL, hR, EL, ER, lim):
    """Interior face: interpolated sigma and E, reduced gradient R, D = c lambda / sigma_f."""
    h = hL + hR
    sig_f = (hL * sigL + hR * sigR) / h
    E_f = (hR * EL + hL * ER) / h
    R = np.abs(ER - EL) / (h * sig_f * E_f)
    return C_LIGHT * lim(R) / sig_f


def boundary_terms(kind, value, ghost, E1, sig1, h1, dS, dt, lim):
    """Diagonal and right-hand-side additions from one side's boundary faces.

    h1 is the distance from the first cell's centre to the boundary face.
      reflecting / axis : no flux.
      Dirichlet face    : E_b = a_R T_b^4 on the face; sigma_f = sigma_1, E_f = E_b,
                          h = h1; W_b = dt dS D / h1; diag += W_b, rhs += W_b E_b.
      Dirichlet ghost   : ghost cell mirrored across the face (centre distance 2 h1),
                          sigma_f = sigma_1, E_f = (E_1 + E_g)/2; rhs += W_b E_g.
      fixed inward flux : rhs += dt dS F_in.
      free streaming    : outward flux c E_1, diag += dt dS c.
      Milne             : E_b = -2/(3 sigma_1) dE/dn on the face (Section 5.2 radiative
                          shock set-up, the blackbody-absorber condition), the
                          outward derivative taken as (E_b - E_1)/h1: E_b = a E_1/(1+a),
                          a = 2/(3 sigma_1 h1); the face's R = |grad E|/(sigma_1 E_b) is
                          3/2 exactly, D = c lambda(3/2)/sigma_1; outward flux
                          D E_1/(h1 (1+a)): diag += dt dS D/(h1 (1+a)).
    Returns (diag_add, rhs_add, W_b, D_b).
    """
    z = np.zeros_like(E1)
    if kind in (REFLECT, AXIS):
        return z, z, z, z
    if kind == DIRICHLET_FACE:
        Eb = A_RAD * value ** 4
        R = np.abs(Eb - E1) / (h1 * sig1 * Eb)
        D = C_LIGHT * lim(R) / sig1
        Wb = dt * dS * D / h1
        return Wb, Wb * Eb, Wb, D
    if kind == DIRICHLET_GHOST:
        Eg = np.asarray(ghost, dtype=np.float64)
        h = 2.0 * h1
        Ef = 0.5 * (E1 + Eg)
        R = np.abs(Eg - E1) / (h * sig1 * Ef)
        D = C_LIGHT * lim(R) / sig1
        Wb = dt * dS * D / h
        return Wb, Wb * Eg, Wb, D
    if kind == FLUX_IN:
        return z, dt * dS * value, z, z
    if kind == FREE_STREAM:
        return dt * dS * C_LIGHT, z, z, z
    if kind == MILNE:
        a = 2.0 / (3.0 * sig1 * h1)
        D = C_LIGHT * lim(np.full_like(sig1, 1.5)) / sig1
        Wb = dt * dS * D / (h1 * (1.0 + a))
        return Wb, z, Wb, D
    raise ValueError("unknown boundary kind")


def advection_volume_term(met: Metrics, E, rho, fx, fy) -> np.ndarray:
    """dV S_adv of every cell (Section 3.2.1 advection term, explicit in time):
    the sum over the cell's faces of +-dS f e_r, inflow through the lower x and
    y faces positive, outflow through the upper ones negative, with f the
    face mass flux (positive along +x / +y) and e_r = E / rho taken from the
    upwind cell.  Reading: at a boundary face the boundary cell's own e_r is
    used for either flow direction (zero-gradient e_r)."""
    E = np.asarray(E, dtype=np.float64)
    er = E / np.asarray(rho, dtype=np.float64)
    fx = np.asarray(fx, dtype=np.float64).reshape(met.ny, met.nx + 1)
    fy = np.asarray(fy, dtype=np.float64).reshape(met.ny + 1, met.nx)
    # e_r of the cells below / above each face, the boundary cell repeated outside
    er_lo_x = np.concatenate([er[:, :1], er], axis=1)
    er_hi_x = np.concatenate([er, er[:, -1:]], axis=1)
    er_lo_y = np.concatenate([er[:1, :], er], axis=0)
    er_hi_y = np.concatenate([er, er[-1:, :]], axis=0)
    tx = met.dSx * fx * np.where(fx >= 0.0, er_lo_x, er_hi_x)  # transport through x faces along +x
    ty = met.dSy * fy * np.where(fy >= 0.0, er_lo_y, er_hi_y)
    return (tx[:, :-1] - tx[:, 1:]) + (ty[:-1, :] - ty[1:, :])


def assemble(geom, xf, yf, E, T, rho, kappa_R, kappa_P, c_v, dt,
             bcs: Sequence[BCSpec], limiter: int = LIMITER_LP, fx=None, fy=None, E_op=None) -> Assembled:
    """Build the volume-weighted, T-eliminated E system of one backward-Euler
    step.  fx [ny][nx+1], fy [ny+1][nx]: face mass fluxes rho v of the
    advection term (None: S_adv = 0), added explicitly as dt dV S_adv.

    E_op: the radiation energy that the interface coefficients D (interior
    and boundary faces) and the advection term are evaluated from; None takes
    E itself.  In the sub-cycled step D and S_adv come from the step's start
    (Section 3.2.1 radiation-subsystem algorithm, steps 1 and 2, taken once),
    while E enters the sub-step's own time derivative."""
    lim = LIMITERS[limiter]
    met = metrics(geom, xf, yf)
    nx, ny = met.nx, met.ny
    E = np.asarray(E, dtype=np.float64).reshape(ny, nx)
    Eo = E if E_op is None else np.asarray(E_op, dtype=np.float64).reshape(ny, nx)
    T = np.asarray(T, dtype=np.float64).reshape(ny, nx)
    rho = np.asarray(rho, dtype=np.float64).reshape(ny, nx)
    kR = np.asarray(kappa_R, dtype=np.float64).reshape(ny, nx)
    kP = np.asarray(kappa_P, dtype=np.float64).reshape(ny, nx)
    cv = np.asarray(c_v, dtype=np.float64).reshape(ny, nx)
    sig = kR * rho

    W_x = np.zeros((ny, nx + 1))
    W_y = np.zeros((ny + 1, nx))
    D_x = np.zeros((ny, nx + 1))
    D_y = np.zeros((ny + 1, nx))
    # interior x faces: between cells i-1 and i, i = 1..nx-1
    if nx > 1:
        hL, hR = met.hLx[:, 1:-1], met.hRx[:, 1:-1]
        D = face_D(sig[:, :-1], sig[:, 1:], hL, hR, Eo[:, :-1], Eo[:, 1:], lim)
        D_x[:, 1:-1] = D
        W_x[:, 1:-1] = dt * met.dSx[:, 1:-1] * D / (hL + hR)
    if ny > 1:
        hL, hR = met.hLy[1:-1, :], met.hRy[1:-1, :]
        D = face_D(sig[:-1, :], sig[1:, :], hL, hR, Eo[:-1, :], Eo[1:, :], lim)
        D_y[1:-1, :] = D
        W_y[1:-1, :] = dt * met.dSy[1:-1, :] * D / (hL + hR)

    bdiag = np.zeros((ny, nx))
    brhs = np.zeros((ny, nx))
    # side order: xlo, xhi, ylo, yhi; ghost arrays run along the side
    sides = [
        (np.s_[:, 0], met.hRx[:, 0], met.dSx[:, 0], (np.s_[:, 0], "x")),
        (np.s_[:, -1], met.hLx[:, -1], met.dSx[:, -1], (np.s_[:, -1], "x")),
        (np.s_[0, :], met.hRy[0, :], met.dSy[0, :], (np.s_[0, :], "y")),
        (np.s_[-1, :], met.hLy[-1, :], met.dSy[-1, :], (np.s_[-1, :], "y")),
    ]
    for b, (cell, h1, dS, (face, ax)) in zip(bcs, sides):
        da, ra, Wb, Db = boundary_terms(b.kind, b.value, b.ghost, Eo[cell], sig[cell], h1, dS, dt, lim)
        bdiag[cell] += da
        brhs[cell] += ra
        if ax == "x":
            W_x[face] = Wb
            D_x[face] = Db
        else:
            W_y[face] = Wb
            D_y[face] = Db

    CV = rho * cv
    beta = kP * rho * C_LIGHT * dt
    X = 4.0 * beta * A_RAD * T ** 3
    f = CV / (CV + X)
    # interior conductances only (boundary faces already in bdiag)
    Wxi = W_x.copy()
    Wxi[:, 0] = 0.0
    Wxi[:, -1] = 0.0
    Wyi = W_y.copy()
    Wyi[0, :] = 0.0
    Wyi[-1, :] = 0.0
    sumW = Wxi[:, :-1] + Wxi[:, 1:] + Wyi[:-1, :] + Wyi[1:, :]
    diag = met.dV * (1.0 + beta * f) + sumW + bdiag
    rhs = met.dV * (E + beta * f * A_RAD * T ** 4) + brhs
    if fx is not None or fy is not None:
        fx = np.zeros((ny, nx + 1)) if fx is None else fx
        fy = np.zeros((ny + 1, nx)) if fy is None else fy
        rhs = rhs + dt * advection_volume_term(met, Eo, rho, fx, fy)
    M = build_matrix(diag, Wxi, Wyi)
    return Assembled(met, W_x, W_y, D_x, D_y, diag, rhs, CV, beta, X, f, bdiag, brhs, M)


def build_matrix(diag, Wxi, Wyi) -> sp.csr_matrix:
    """Symmetric 5-point matrix with the given diagonal and interior face conductances."""
    ny, nx = diag.shape
    n = nx * ny
    idx = np.arange(n).reshape(ny, nx)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [diag.ravel()]
    if nx > 1:
        w = Wxi[:, 1:-1].ravel()
        a, b = idx[:, :-1].ravel(), idx[:, 1:].ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-w, -w]
    if ny > 1:
        w = Wyi[1:-1, :].ravel()
        a, b = idx[:-1, :].ravel(), idx[1:, :].ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-w, -w]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


# ---------------------------------------------------------------------------
# solve, gas update, diagnostics
# ---------------------------------------------------------------------------

def solve(A: Assembled) -> np.ndarray:
    """E^{n+1}: the solution of the SPD system M E = rhs (Section 3.2.1 step 6),
    to rounding.

    A sparse direct factorisation (SuperLU) alone leaves a Jacobi-scaled
    residual near 1e-10 on optically thin spherical shells, where the face
    conductances exceed the cell masses by ten orders of magnitude.  The
    solution is therefore refined with the same factors: r = rhs - M E is
    formed in extended precision (x87 long double, 64-bit significand), then
    E += LU^-1 r, until the scaled residual stops falling (at most 8 passes).
    """
    ny, nx = A.diag.shape
    lu = spla.splu(A.M.tocsc(), permc_spec="COLAMD")
    b = A.rhs.ravel()
    x = lu.solve(b)
    Ml = A.M.astype(np.longdouble)
    bl = b.astype(np.longdouble)
    s = 1.0 / np.sqrt(A.diag.ravel())
    bn = np.linalg.norm(s * b)
    best = np.inf
    for _ in range(8):
        r = bl - Ml @ x.astype(np.longdouble)
        rn = np.linalg.norm(s * r.astype(np.float64)) / bn if bn > 0 else 0.0
        if not rn < 0.5 * best:
            break
        best = rn
        x = x + lu.solve(r.astype(np.float64))
    return x.reshape(ny, nx)


def gas_update(A: Assembled, T, E_new):
    """T^{n+1} from the psi row: (C_V T + 3 beta a_R T^4 + beta E^{n+1}) / (C_V + 4 beta a_R T^3)."""
    T = np.asarray(T, dtype=np.float64).reshape(A.diag.shape)
    return (A.CV * T + 3.0 * A.beta * A_RAD * T ** 4 + A.beta * E_new) / (A.CV + A.X)


def residual_rowform(A: Assembled, E_new) -> float:
    """||(rhs - M E)/dV||_2 / ||rhs/dV||_2: the per-volume (phi-row) form of the stop rule."""
    E_new = np.asarray(E_new, dtype=np.float64).ravel()
    r = (A.rhs.ravel() - A.M @ E_new) / A.met.dV.ravel()
    return float(np.linalg.norm(r) / np.linalg.norm(A.rhs.ravel() / A.met.dV.ravel()))


def residual_scaled(A: Assembled, E_new) -> float:
    """||S (rhs - M E)||_2 / ||S rhs||_2 with S = diag(M)^(-1/2)."""
    E_new = np.asarray(E_new, dtype=np.float64).ravel()
    s = 1.0 / np.sqrt(A.diag.ravel())
    r = s * (A.rhs.ravel() - A.M @ E_new)
    return float(np.linalg.norm(r) / np.linalg.norm(s * A.rhs.ravel()))


def total_energy(A: Assembled, E, T) -> float:
    """Sum over cells of dV (E + C_V T): radiation plus (linearised) gas energy."""
    return float(np.sum(A.met.dV * (np.asarray(E).reshape(A.diag.shape) + A.CV * np.asarray(T).reshape(A.diag.shape))))


def boundary_energy_input(geom, A: Assembled, bcs: Sequence[BCSpec], E_new, dt) -> float:
    """Energy that entered through the boundary faces during the step (erg, 2 pi dropped)."""
    E_new = np.asarray(E_new).reshape(A.diag.shape)
    met = A.met
    total = 0.0
    cells = [np.s_[:, 0], np.s_[:, -1], np.s_[0, :], np.s_[-1, :]]
    faces = [(A.W_x, np.s_[:, 0], met.dSx[:, 0]), (A.W_x, np.s_[:, -1], met.dSx[:, -1]),
             (A.W_y, np.s_[0, :], met.dSy[0, :]), (A.W_y, np.s_[-1, :], met.dSy[-1, :])]
    for b, cell, (W, face, dS) in zip(bcs, cells, faces):
        E1 = E_new[cell]
        if b.kind == DIRICHLET_FACE:
            total += float(np.sum(W[face] * (A_RAD * b.value ** 4 - E1)))
        elif b.kind == DIRICHLET_GHOST:
            total += float(np.sum(W[face] * (np.asarray(b.ghost) - E1)))
        elif b.kind == FLUX_IN:
            total += float(np.sum(dt * dS * b.value))
        elif b.kind == FREE_STREAM:
            total -= float(np.sum(dt * dS * C_LIGHT * E1))
    return total


def face_fluxes(A: Assembled, E_old, E_new, sig, dt, bcs: Sequence[BCSpec], limiter: int = LIMITER_LP):
    """Radiative flux through every face after a step (Section 3.2.1 flux
    formula, one sub-step), positive along +x / +y: Fx [ny][nx+1], Fy [ny+1][nx].
    An interior face carries W (E_lo - E_hi) / (dt dS) = -D (E_hi - E_lo) / h
    with the step's conductance W; a boundary face the outward flux its side's
    boundary terms put in the rows, (da E_1 - ra) / (dt dS) (da, ra from
    ``boundary_terms`` with the step's E^n), sign-flipped on the lower sides.
    Faces of zero area (the axis) carry none."""
    met = A.met
    lim = LIMITERS[limiter]
    ny, nx = met.ny, met.nx
    E_old = np.asarray(E_old, dtype=np.float64).reshape(ny, nx)
    E_new = np.asarray(E_new, dtype=np.float64).reshape(ny, nx)
    sig = np.asarray(sig, dtype=np.float64).reshape(ny, nx)
    Fx = np.zeros((ny, nx + 1))
    Fy = np.zeros((ny + 1, nx))
    Fx[:, 1:-1] = A.W_x[:, 1:-1] * (E_new[:, :-1] - E_new[:, 1:]) / (dt * met.dSx[:, 1:-1])
    Fy[1:-1, :] = A.W_y[1:-1, :] * (E_new[:-1, :] - E_new[1:, :]) / (dt * met.dSy[1:-1, :])
    sides = [(np.s_[:, 0], met.hRx[:, 0], met.dSx[:, 0], Fx, np.s_[:, 0], -1.0),
             (np.s_[:, -1], met.hLx[:, -1], met.dSx[:, -1], Fx, np.s_[:, -1], 1.0),
             (np.s_[0, :], met.hRy[0, :], met.dSy[0, :], Fy, np.s_[0, :], -1.0),
             (np.s_[-1, :], met.hLy[-1, :], met.dSy[-1, :], Fy, np.s_[-1, :], 1.0)]
    for b, (cell, h1, dS, F, face, sgn) in zip(bcs, sides):
        da, ra, _, _ = boundary_terms(b.kind, b.value, b.ghost, E_old[cell], sig[cell], h1, dS, dt, lim)
        with np.errstate(divide="ignore", invalid="ignore"):
            out = np.where(dS > 0.0, (da * E_new[cell] - ra) / (dt * dS), 0.0)
        F[face] = sgn * out
    return Fx, Fy


def interface_flux_x(A: Assembled, E_new):
    """F at interior x faces, -D (E_R - E_L)/h with D at level n (Section 3.2.1, flux formula, one sub-step)."""
    E_new = np.asarray(E_new).reshape(A.diag.shape)
    h = A.met.hLx[:, 1:-1] + A.met.hRx[:, 1:-1]
    return -A.D_x[:, 1:-1] * (E_new[:, 1:] - E_new[:, :-1]) / h


@dataclasses.dataclass
class StepResult:
    E: np.ndarray
    T: np.ndarray
    A: Assembled


def step(geom, xf, yf, E, T, rho, kappa_R, kappa_P, c_v, dt, bcs, limiter=LIMITER_LP, fx=None,
         fy=None) -> StepResult:
    """One implicit radiation step: assemble, solve, gas update."""
    A = assemble(geom, xf, yf, E, T, rho, kappa_R, kappa_P, c_v, dt, bcs, limiter, fx, fy)
    E_new = solve(A)
    T_new = gas_update(A, T, E_new)
    return StepResult(E_new, T_new, A)


def bcs_from_problem(prob) -> List[BCSpec]:
    """Translate a fld_workloads.Problem boundary list (with packed ghosts) to BCSpec."""
    out = []
    nx, ny = prob.nx, prob.ny
    offs = {0: (0, ny), 1: (ny, 2 * ny), 2: (2 * ny, 2 * ny + nx), 3: (2 * ny + nx, 2 * ny + 2 * nx)}
    for s, b in enumerate(prob.bc):
        g = None
        if b.kind == DIRICHLET_GHOST:
            lo, hi = offs[s]
            g = np.asarray(prob.ghost_E[lo:hi], dtype=np.float64)
        out.append(BCSpec(b.kind, b.value, g))
    return out


def step_problem(prob, E=None, T=None, limiter=LIMITER_LP, fx=None, fy=None) -> StepResult:
    E = prob.E if E is None else E
    T = prob.T if T is None else T
    return step(prob.geom, prob.x_faces, prob.y_faces, E, T, prob.rho, prob.kappa_R, prob.kappa_P,
                prob.c_v, prob.dt, bcs_from_problem(prob), limiter, fx, fy)


def assemble_problem(prob, E=None, T=None, limiter=LIMITER_LP) -> Assembled:
    E = prob.E if E is None else E
    T = prob.T if T is None else T
    return assemble(prob.geom, prob.x_faces, prob.y_faces, E, T, prob.rho, prob.kappa_R, prob.kappa_P,
                    prob.c_v, prob.dt, bcs_from_problem(prob), limiter)
