"""The paper's coupled (E, T) linear system, built literally from phi/psi.

TEST INFRASTRUCTURE ONLY (see fld_oracle.py).  This is a second, independent
route to the same backward-Euler step for tiny grids: instead of eliminating
T and solving the volume-weighted E system, it writes out the 2 N1 N2 unknowns
of Section 3.2.1 (two equations per cell, phi row for E and psi row for T)
with pure-Python loops, and solves the dense system with LAPACK.

Coefficients (Section 3.2.1, coefficient list; D > 0 and the exchange sign
of Section 2, kappa_e = kappa_P):

  phi_1, phi_3, phi_7, phi_9 = -alpha g D  for the S, W, E, N neighbour,
      alpha = dt / (centre distance), g = dS / dV,
  phi_5  = 1 - phi_1 - phi_3 - phi_7 - phi_9 + beta_P,
  phi_6  = -4 beta_e a_R T^3,
  phi_11 = E^n - 3 beta_e a_R T^4,
  psi_5  = -beta_P,  psi_6 = C_V + 4 beta_e a_R T^3,
  psi_11 = C_V T^n + 3 beta_e a_R T^4.

Boundary faces enter the phi row divided by the cell volume.  Face D values,
boundary additions and metrics come from fld_oracle (pinned separately); the
elimination of T, the volume weighting and the gas update are what this
route checks.
"""
from __future__ import annotations

import numpy as np

from .fld_oracle import A_RAD, C_LIGHT, Assembled


def coupled_system(A: Assembled, E, T, rho, kappa_P, c_v, dt):
    met = A.met
    nx, ny = met.nx, met.ny
    E = np.asarray(E, dtype=np.float64).reshape(ny, nx)
    T = np.asarray(T, dtype=np.float64).reshape(ny, nx)
    rho = np.asarray(rho, dtype=np.float64).reshape(ny, nx)
    kP = np.asarray(kappa_P, dtype=np.float64).reshape(ny, nx)
    cv = np.asarray(c_v, dtype=np.float64).reshape(ny, nx)
    n = nx * ny
    Amat = np.zeros((2 * n, 2 * n))
    b = np.zeros(2 * n)

    def e(i, j):
        return 2 * (j * nx + i)

    for j in range(ny):
        for i in range(nx):
            dV = met.dV[j, i]
            beta = kP[j, i] * rho[j, i] * C_LIGHT * dt
            CV = rho[j, i] * cv[j, i]
            Tn = T[j, i]
            off = {}
            if j > 0:    # south face j-1/2
                h = met.hLy[j, i] + met.hRy[j, i]
                off[(i, j - 1)] = -(dt / h) * (met.dSy[j, i] / dV) * A.D_y[j, i]
            if i > 0:    # west face i-1/2
                h = met.hLx[j, i] + met.hRx[j, i]
                off[(i - 1, j)] = -(dt / h) * (met.dSx[j, i] / dV) * A.D_x[j, i]
            if i < nx - 1:  # east face i+1/2
                h = met.hLx[j, i + 1] + met.hRx[j, i + 1]
                off[(i + 1, j)] = -(dt / h) * (met.dSx[j, i + 1] / dV) * A.D_x[j, i + 1]
            if j < ny - 1:  # north face j+1/2
                h = met.hLy[j + 1, i] + met.hRy[j + 1, i]
                off[(i, j + 1)] = -(dt / h) * (met.dSy[j + 1, i] / dV) * A.D_y[j + 1, i]
            row_E = e(i, j)
            row_T = row_E + 1
            phi5 = 1.0 - sum(off.values()) + beta + A.bdiag[j, i] / dV
            for (ii, jj), v in off.items():
                Amat[row_E, e(ii, jj)] = v
            Amat[row_E, row_E] = phi5
            Amat[row_E, row_T] = -4.0 * beta * A_RAD * Tn ** 3
            b[row_E] = E[j, i] - 3.0 * beta * A_RAD * Tn ** 4 + A.brhs[j, i] / dV
            Amat[row_T, row_E] = -beta
            Amat[row_T, row_T] = CV + 4.0 * beta * A_RAD * Tn ** 3
            b[row_T] = CV * Tn + 3.0 * beta * A_RAD * Tn ** 4
    return Amat, b


def solve_coupled(A: Assembled, E, T, rho, kappa_P, c_v, dt):
    Amat, b = coupled_system(A, E, T, rho, kappa_P, c_v, dt)
    x = np.linalg.solve(Amat, b)
    ny, nx = A.diag.shape
    return x[0::2].reshape(ny, nx), x[1::2].reshape(ny, nx)
