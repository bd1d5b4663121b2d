"""FP64 CPU oracle for one implicit FLD radiation step on a statically refined
block forest, solved as one matrix across refinement levels (Section 3.2.2,
the multilevel linear system with five neighbours for a coarse cell at a
level jump; Section 4, radiation communications).

TEST INFRASTRUCTURE ONLY, like ``fld_oracle``: only the tests, the smoke check
and the benchmark's CPU leg may use it.

The forest is a 2D Cartesian domain covered by leaf blocks.  Block b has a
refinement level L_b (cell size dx0 / 2^L, dy0 / 2^L) and covers the cells
(i0 .. i0+nx-1, j0 .. j0+ny-1) of its level's index space; cells are numbered
block after block, each block row-major.  Neighbouring leaf cells differ by at
most one level (2:1 balance); a fine block covers whole cells of the coarser
level (even i0, j0, nx, ny).

Every face between two leaf cells carries one conductance used by both rows
(so the matrix is symmetric and the flux leaving one cell enters the other):
  * same level: the uniform-grid face (Section 3.2.1): sigma and E
    interpolated linearly between the two centres, R from the two-point
    normal difference, D = c lambda(R) / sigma_f, W = dt dS D / h;
  * level jump: each fine face (half of the coarse cell's side) couples the
    fine cell to the coarse cell directly, with the fine face's area and the
    normal distance of the two centres, h = dx_fine / 2 + dx_coarse / 2; the
    face's sigma, E and gradient are interpolated linearly along that
    distance, exactly as on a uniform face.  The coarse cell therefore sees
    two neighbours on that side, each through its own D (the paper's coarse
    cell with five neighbours), and the flux through its side is the sum of
    the two fine faces' fluxes.
Readings (the figure that fixes the interpolation points is not in the text):
the interpolation runs along the normal through the two centres, the coarse
centre's lateral offset of half a fine cell being neglected, i.e. the
two-point flux of the uniform grid with unequal centre distances.

Cells, the T elimination, the gas update and the boundary faces on the domain
sides are those of ``fld_oracle`` (reflecting, Dirichlet face, fixed inward
flux, free streaming).  The system is solved directly (SuperLU with
extended-precision refinement).

Parity status: pinned by tests/test_oracle_forest.py: a forest of level-0
blocks equals the uniform-grid oracle on their union; symmetry and diagonal
dominance; the equilibrium fixed point; conservation of total energy with
every domain boundary kind; a steady linear profile held exactly across level
jumps (which fixes the jump distance and the face areas); every cell's
balance with the exported face fluxes; and convergence of a spreading
Gaussian on refined forests to the analytic solution.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Sequence, Tuple

import numpy as np
import scipy.sparse as sp

from . import fld_oracle as O


@dataclasses.dataclass
class Block:
    level: int
    i0: int
    j0: int
    nx: int
    ny: int


@dataclasses.dataclass
class Forest:
    """Leaf cells and faces of a block forest."""
    n: int
    level: np.ndarray      # per cell
    xc: np.ndarray         # centre
    yc: np.ndarray
    dx: np.ndarray         # cell size
    dy: np.ndarray
    dV: np.ndarray
    fa: np.ndarray         # faces: lower / left cell
    fb: np.ndarray         # upper / right cell
    farea: np.ndarray
    fha: np.ndarray        # distance from cell a's centre to the face (normal)
    fhb: np.ndarray
    faxis: np.ndarray      # 0: x face, 1: y face
    bcell: np.ndarray      # domain-boundary faces: cell
    bside: np.ndarray      # side 0..3 (xlo, xhi, ylo, yhi)
    barea: np.ndarray
    bh: np.ndarray         # centre to boundary face


def build(blocks: Sequence[Block], dx0: float, dy0: float, NX0: int, NY0: int) -> Forest:
    """Leaf cells and faces of a forest covering [0, NX0 dx0] x [0, NY0 dy0]."""
    cells: Dict[Tuple[int, int, int], int] = {}
    lev, ci, cj = [], [], []
    for b in blocks:
        for j in range(b.j0, b.j0 + b.ny):
            for i in range(b.i0, b.i0 + b.nx):
                key = (b.level, i, j)
                if key in cells:
                    raise ValueError("overlapping blocks")
                cells[key] = len(lev)
                lev.append(b.level)
                ci.append(i)
                cj.append(j)
    lev = np.array(lev)
    ci = np.array(ci)
    cj = np.array(cj)
    n = lev.size
    dx = dx0 / 2.0 ** lev
    dy = dy0 / 2.0 ** lev
    xc = (ci + 0.5) * dx
    yc = (cj + 0.5) * dy
    # coverage: total area equals the domain's
    if not np.isclose(np.sum(dx * dy), NX0 * dx0 * NY0 * dy0, rtol=1e-12):
        raise ValueError("blocks do not cover the domain")
    fa, fb, farea, fha, fhb, fax = [], [], [], [], [], []
    bc_cell, bc_side, bc_area, bc_h = [], [], [], []

    def lookup(L, i, j):
        return cells.get((L, i, j))

    for c in range(n):
        L, i, j = int(lev[c]), int(ci[c]), int(cj[c])
        nxL, nyL = NX0 * 2 ** L, NY0 * 2 ** L
        for side, (di, dj) in enumerate(((-1, 0), (1, 0), (0, -1), (0, 1))):
            axis = 0 if side < 2 else 1
            ii, jj = i + di, j + dj
            if not (0 <= ii < nxL and 0 <= jj < nyL):
                bc_cell.append(c)
                bc_side.append(side)
                bc_area.append(dy[c] if axis == 0 else dx[c])
                bc_h.append(0.5 * (dx[c] if axis == 0 else dy[c]))
                continue
            same = lookup(L, ii, jj)
            coarse = lookup(L - 1, ii // 2, jj // 2) if L > 0 else None
            if same is not None:
                if side in (1, 3):  # each same-level face once, from its lower cell
                    fa.append(c)
                    fb.append(same)
                    farea.append(dy[c] if axis == 0 else dx[c])
                    h = 0.5 * (dx[c] if axis == 0 else dy[c])
                    fha.append(h)
                    fhb.append(h)
                    fax.append(axis)
            elif coarse is not None:
                # level jump seen from the fine cell: one fine face to the coarse cell
                a, b = (coarse, c) if side in (0, 2) else (c, coarse)
                hf = 0.5 * (dx[c] if axis == 0 else dy[c])
                hc = 0.5 * (dx[coarse] if axis == 0 else dy[coarse])
                fa.append(a)
                fb.append(b)
                farea.append(dy[c] if axis == 0 else dx[c])
                fha.append(hc if a == coarse else hf)
                fhb.append(hf if a == coarse else hc)
                fax.append(axis)
            else:
                # finer neighbours: their faces are added from the fine side
                f0 = lookup(L + 1, 2 * ii + (1 if di < 0 else 0) if axis == 0 else 2 * ii,
                            2 * jj + (1 if dj < 0 else 0) if axis == 1 else 2 * jj)
                if f0 is None:
                    raise ValueError(f"cell {c} (level {L}, {i}, {j}) has no neighbour on side {side}: "
                                     "the forest is not 2:1 balanced or leaves a hole")
    return Forest(n, lev, xc, yc, dx, dy, dx * dy, np.array(fa, dtype=np.int64), np.array(fb, dtype=np.int64),
                  np.array(farea), np.array(fha), np.array(fhb), np.array(fax), np.array(bc_cell, dtype=np.int64),
                  np.array(bc_side), np.array(bc_area), np.array(bc_h))


@dataclasses.dataclass
class ForestSystem:
    W: np.ndarray          # conductance of every interior face
    bdiag: np.ndarray      # per cell, boundary terms
    brhs: np.ndarray
    bface_d: np.ndarray    # per boundary face: its diagonal and right-hand-side terms
    bface_r: np.ndarray
    CV: np.ndarray
    beta: np.ndarray
    X: np.ndarray
    diag: np.ndarray
    rhs: np.ndarray
    M: sp.csr_matrix


def assemble(F: Forest, E, T, rho, kappa_R, kappa_P, c_v, dt, bcs: Sequence[O.BCSpec],
             limiter: int = O.LIMITER_LP) -> ForestSystem:
    """The volume-weighted, T-eliminated system on the forest (the uniform
    grid's cell rows, one conductance per leaf face)."""
    lim = O.LIMITERS[limiter]
    E, T, rho = (np.asarray(a, dtype=np.float64).ravel() for a in (E, T, rho))
    kR, kP, cv = (np.asarray(a, dtype=np.float64).ravel() for a in (kappa_R, kappa_P, c_v))
    sig = kR * rho
    a, b = F.fa, F.fb
    D = O.face_D(sig[a], sig[b], F.fha, F.fhb, E[a], E[b], lim)
    W = dt * F.farea * D / (F.fha + F.fhb)
    bdiag = np.zeros(F.n)
    brhs = np.zeros(F.n)
    bd = np.zeros(F.bcell.size)
    br = np.zeros(F.bcell.size)
    for s in range(4):
        sel = np.nonzero(F.bside == s)[0]
        if sel.size == 0:
            continue
        c = F.bcell[sel]
        spec = bcs[s]
        if spec.kind == O.DIRICHLET_GHOST:
            raise ValueError("the forest takes reflecting, Dirichlet-face, inflow and free-streaming sides")
        d, r, _, _ = O.boundary_terms(spec.kind, spec.value, None, E[c], sig[c], F.bh[sel], F.barea[sel], dt, lim)
        bd[sel] = d
        br[sel] = r
        np.add.at(bdiag, c, d)
        np.add.at(brhs, c, r)
    CV = rho * cv
    beta = kP * rho * O.C_LIGHT * dt
    X = 4.0 * beta * O.A_RAD * T ** 3
    f = CV / (CV + X)
    sumW = np.zeros(F.n)
    np.add.at(sumW, a, W)
    np.add.at(sumW, b, W)
    diag = F.dV * (1.0 + beta * f) + sumW + bdiag
    rhs = F.dV * (E + beta * f * O.A_RAD * T ** 4) + brhs
    M = sp.csr_matrix((np.concatenate([diag, -W, -W]),
                       (np.concatenate([np.arange(F.n), a, b]), np.concatenate([np.arange(F.n), b, a]))),
                      shape=(F.n, F.n))
    return ForestSystem(W, bdiag, brhs, bd, br, CV, beta, X, diag, rhs, M)


@dataclasses.dataclass
class ForestStep:
    E: np.ndarray
    T: np.ndarray
    S: ForestSystem


def step(F: Forest, E, T, rho, kappa_R, kappa_P, c_v, dt, bcs, limiter=O.LIMITER_LP) -> ForestStep:
    S = assemble(F, E, T, rho, kappa_R, kappa_P, c_v, dt, bcs, limiter)
    A = O.Assembled(None, None, None, None, None, S.diag.reshape(1, -1), S.rhs.reshape(1, -1), S.CV, S.beta, S.X,
                    None, None, None, S.M)
    E_new = O.solve(A).ravel()
    T = np.asarray(T, dtype=np.float64).ravel()
    T_new = (S.CV * T + 3.0 * S.beta * O.A_RAD * T ** 4 + S.beta * E_new) / (S.CV + S.X)
    return ForestStep(E_new, T_new, S)


def face_fluxes(F: Forest, S: ForestSystem, E_new, dt):
    """Flux through every interior face (from cell a to cell b, along +x / +y)
    and every boundary face (outward), after a step."""
    E_new = np.asarray(E_new, dtype=np.float64).ravel()
    Fi = S.W * (E_new[F.fa] - E_new[F.fb]) / (dt * F.farea)
    Fb = (S.bface_d * E_new[F.bcell] - S.bface_r) / (dt * F.barea)
    return Fi, Fb
