"""Pins for the diffusion operator (Section 2 FLD closure, Section 3.2.1 face
coefficients and geometric factors, Section 5.2.2 diffusion test).

* The worked numbers of the paper's diffusion test (golden/e4_diffusion.txt):
  the thick-limit D = c/(3 rho kappa_R) must reproduce l_diff = sqrt(4 D t)
  = 0.498 cm, which fixes the factor 3.
* The analytic spreading Gaussian in 1D and 2D (no gas coupling): small error,
  and first-order in the time step (backward Euler).
* Layered steady states with the pure-diffusion limiter: the two-point flux
  with distance-weighted interface opacity is exact for cell-wise constant
  opacity on a non-uniform grid, so the discrete steady state equals the
  analytic one at cell centres, for Dirichlet-face, Dirichlet-ghost,
  inward-flux and free-streaming boundaries.
* Spherical geometry: the radial steady state E = E_b + 3 sigma F r_out^2/c
  (1/r_in - 1/r) and the decay of the cos(theta) mode on a thin shell,
  both converging at second order in the grid spacing.
"""
import os

import numpy as np
import pytest

from oracle import fld_oracle as O
import fld_workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "e4_diffusion.txt")


def golden():
    out = {}
    for line in open(GOLD):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def test_e4_worked_numbers_pin_thick_diffusion_coefficient():
    g = golden()
    sig = g["rho_kappa_R_per_cm"]
    D = O.face_D(np.array([sig]), np.array([sig]), np.array([0.5]), np.array([0.5]),
                 np.array([1.0]), np.array([1.0 + 1e-9]), O.limiter_lp)[0]
    assert round(np.sqrt(4.0 * D * g["t_end_s"]), 3) == g["l_diff_cm"]
    assert round(g["v_cm_per_s"] * g["t_end_s"], 2) == g["l_dyn_cm"]


def gaussian_1d(x, t, D, E0):
    return 1.0 + E0 / np.sqrt(4.0 * np.pi * D * t) * np.exp(-x * x / (4.0 * D * t))


def run_1d(nsteps, g):
    n = int(g["ncells"])
    xf = np.linspace(g["domain_lo_cm"], g["domain_hi_cm"], n + 1)
    yf = np.array([0.0, 1.0])
    xc = 0.5 * (xf[1:] + xf[:-1])
    sig = g["rho_kappa_R_per_cm"]
    D = O.C_LIGHT / (3.0 * sig)
    t0 = g["t_end_s"]
    t1 = 2.0 * t0
    E = gaussian_1d(xc, t0, D, g["E0_erg"])[None, :]
    shape = E.shape
    dt = (t1 - t0) / nsteps
    for _ in range(nsteps):
        res = O.step(O.CARTESIAN, xf, yf, E, np.ones(shape), np.ones(shape), np.full(shape, sig),
                     np.zeros(shape), np.ones(shape), dt, [O.BCSpec()] * 4)
        E = res.E
    exact = gaussian_1d(xc, t1, D, g["E0_erg"])
    return np.max(np.abs(E[0] - exact)) / exact.max()


def test_gaussian_1d_first_order_in_time():
    g = golden()
    e1, e2 = run_1d(10, g), run_1d(20, g)
    assert e2 < 0.02
    assert 1.7 < e1 / e2 < 2.3, (e1, e2)


def run_2d(nsteps, n=96):
    L = 1.0
    xf = np.linspace(-L, L, n + 1)
    xc = 0.5 * (xf[1:] + xf[:-1])
    X, Y = np.meshgrid(xc, xc)
    sig = 1e9
    D = O.C_LIGHT / (3.0 * sig)
    t0 = (0.15 ** 2) / (4.0 * D)
    t1 = 2.0 * t0

    def exact(t):
        return 1.0 + 1e3 / (4.0 * np.pi * D * t) * np.exp(-(X * X + Y * Y) / (4.0 * D * t))

    E = exact(t0)
    shape = E.shape
    dt = (t1 - t0) / nsteps
    for _ in range(nsteps):
        E = O.step(O.CARTESIAN, xf, xf, E, np.ones(shape), np.ones(shape), np.full(shape, sig),
                   np.zeros(shape), np.ones(shape), dt, [O.BCSpec()] * 4).E
    ex = exact(t1)
    return np.max(np.abs(E - ex)) / ex.max()


def test_gaussian_2d_first_order_in_time():
    e1, e2 = run_2d(8), run_2d(16)
    assert e2 < 0.03
    assert 1.6 < e1 / e2 < 2.4, (e1, e2)


def layered(nx=23, ny=3, seed=7):
    rng = np.random.default_rng(seed)
    xf = np.concatenate([[0.0], np.cumsum(rng.uniform(0.5, 2.0, nx))])
    yf = np.linspace(0.0, 1.0, ny + 1)
    sig_x = np.exp(rng.uniform(-3, 3, nx))
    xc = 0.5 * (xf[1:] + xf[:-1])
    return xf, yf, xc, sig_x


def steady_check(xf, yf, E_exact, sig_x, bcs, dt=1.0):
    ny, nx = yf.size - 1, xf.size - 1
    E = np.broadcast_to(E_exact[None, :], (ny, nx)).copy()
    ones = np.ones((ny, nx))
    sig = np.broadcast_to(sig_x[None, :], (ny, nx)).copy()
    A = O.assemble(O.CARTESIAN, xf, yf, E, ones * 300.0, ones, sig, 0.0 * ones, ones, dt, bcs,
                   limiter=O.LIMITER_DIFFUSION)
    r = A.rhs.ravel() - A.M @ E.ravel()
    scale = np.abs(A.diag.ravel() * E.ravel()).max()
    assert np.max(np.abs(r)) < 1e-13 * scale
    E1 = O.solve(A)
    np.testing.assert_allclose(E1, E, rtol=1e-9)


def test_layered_steady_state_dirichlet_face_and_flux_in():
    xf, yf, xc, sig = layered()
    Eb, Fin = 2.0, 3e10
    # E rises from x_lo: E(x) = E_b + (3 F / c) * optical depth from x_lo
    tau = np.concatenate([[sig[0] * (xc[0] - xf[0])],
                          sig[:-1] * (xf[1:-1] - xc[:-1]) + sig[1:] * (xc[1:] - xf[1:-1])])
    E = Eb + 3.0 * Fin / O.C_LIGHT * np.cumsum(tau)
    Tb = (Eb / O.A_RAD) ** 0.25
    steady_check(xf, yf, E, sig, [O.BCSpec(O.DIRICHLET_FACE, Tb), O.BCSpec(O.FLUX_IN, Fin), O.BCSpec(), O.BCSpec()])


def test_layered_steady_state_dirichlet_ghost():
    xf, yf, xc, sig = layered(seed=8)
    Eg, Fin = 5.0, 1e10
    h1 = xc[0] - xf[0]
    tau = np.concatenate([[sig[0] * 2.0 * h1],  # ghost centre mirrored across the face, opacity of cell 1
                          sig[:-1] * (xf[1:-1] - xc[:-1]) + sig[1:] * (xc[1:] - xf[1:-1])])
    E = Eg + 3.0 * Fin / O.C_LIGHT * np.cumsum(tau)
    ny = yf.size - 1
    steady_check(xf, yf, E, sig, [O.BCSpec(O.DIRICHLET_GHOST, 0.0, np.full(ny, Eg)), O.BCSpec(O.FLUX_IN, Fin),
                                  O.BCSpec(), O.BCSpec()])


def test_layered_steady_state_free_streaming_outflow():
    xf, yf, xc, sig = layered(seed=9)
    Fin = 4e10
    # flux F_in flows in at x_lo and leaves at x_hi as c E_N
    EN = Fin / O.C_LIGHT
    tau_between = sig[:-1] * (xf[1:-1] - xc[:-1]) + sig[1:] * (xc[1:] - xf[1:-1])
    drop = 3.0 * Fin / O.C_LIGHT * tau_between
    E = EN + np.concatenate([np.cumsum(drop[::-1])[::-1], [0.0]])
    steady_check(xf, yf, E, sig, [O.BCSpec(O.FLUX_IN, Fin), O.BCSpec(O.FREE_STREAM), O.BCSpec(), O.BCSpec()])


def radial_error(n):
    r_in, r_out = 1.0, 3.0
    xf = np.linspace(r_in, r_out, n + 1)
    yf = np.linspace(0.0, np.pi, 4)
    sig, Eb, Fin = 2.0, 1.0, 1e10
    m = O.metrics(O.SPHERICAL, xf, yf)
    rc = m.hLx[0, 1:] * 0 + (xf[:-1] + m.hRx[0, :-1])  # volume centres
    exact = Eb + 3.0 * sig * Fin * r_out ** 2 / O.C_LIGHT * (1.0 / r_in - 1.0 / rc)
    ny = yf.size - 1
    E = np.broadcast_to(exact[None, :], (ny, n)).copy()
    ones = np.ones((ny, n))
    bcs = [O.BCSpec(O.DIRICHLET_FACE, (Eb / O.A_RAD) ** 0.25), O.BCSpec(O.FLUX_IN, Fin),
           O.BCSpec(O.AXIS), O.BCSpec(O.AXIS)]
    A = O.assemble(O.SPHERICAL, xf, yf, E, ones, ones, ones * sig, 0 * ones, ones, 1e30, bcs,
                   limiter=O.LIMITER_DIFFUSION)
    E1 = O.solve(A)
    return np.max(np.abs(E1 - E)) / (exact.max() - Eb)


def test_spherical_radial_steady_state_second_order():
    e = [radial_error(n) for n in (16, 32, 64)]
    assert e[2] < 2e-3
    assert 3.3 < e[0] / e[1] < 4.7 and 3.3 < e[1] / e[2] < 4.7, e


def theta_mode_error(ny):
    r0 = 2.5
    xf = np.array([r0, r0 * 1.0001])
    yf = W.theta_faces(ny)
    sig, eps, dt = 1.0, 1e-3, 2e-11 * r0 * r0
    D = O.C_LIGHT / (3.0 * sig)
    m = O.metrics(O.SPHERICAL, xf, yf)
    rc = xf[0] + m.hRx[0, 0]
    tc = yf[:-1] + m.hRy[:-1, 0] / rc
    E = (1.0 + eps * np.cos(tc))[:, None]
    ones = np.ones_like(E)
    bcs = [O.BCSpec(), O.BCSpec(), O.BCSpec(O.AXIS), O.BCSpec(O.AXIS)]
    E1 = O.step(O.SPHERICAL, xf, yf, E, ones, ones, ones * sig, 0 * ones, ones, dt, bcs,
                limiter=O.LIMITER_DIFFUSION).E
    g = 1.0 / (1.0 + 2.0 * D * dt / rc ** 2)
    return np.max(np.abs((E1[:, 0] - 1.0) - eps * g * np.cos(tc))) / eps, g


def test_spherical_theta_mode_decay_second_order():
    (e1, g), (e2, _), (e3, _) = theta_mode_error(64), theta_mode_error(128), theta_mode_error(256)
    assert g < 0.9  # the step really decays the mode
    assert e3 < 5e-5
    # second order away from the poles; the pole cells pull the observed rate
    # slightly below 4 at these resolutions (3.15, 3.30, 3.40 for 64..512)
    assert 3.0 < e1 / e2 < 4.7 and 3.0 < e2 / e3 < 4.7, (e1, e2, e3)
