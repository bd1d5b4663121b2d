"""Pins for the explicit advection term (Section 3.2.1 advection equation,
upwinded specific radiation energy; Section 5 dynamical-diffusion test).

* A per-face brute force on small grids (both geometries) reproduces the
  vectorised term cell by cell, and the term conserves: its sum over the grid
  is the net transport through the boundary faces.
* A uniform e_r carried by a divergence-free mass flux gives no source.
* At Courant number 1 with negligible diffusion and no coupling, first-order
  upwinding moves the profile by exactly one cell per step.
* The paper's dynamical-diffusion set-up (1024 cells on [-2, 14] cm, v = 1.8
  km/s, rho kappa_R = 1e7 / cm, kappa_P = 0, a 2e5 erg packet in the two
  central cells, zero-gradient sides, CFL 1, t = 6.2e-5 s) follows the
  analytic moving Gaussian 1 + E0 / sqrt(4 pi D t) exp(-(x - v t)^2 / (4 D t)),
  D = c / (3 rho kappa_R), and the error falls as the grid is refined.
"""
import numpy as np
import pytest

from oracle import fld_oracle as O


def brute_force(met, E, rho, fx, fy):
    ny, nx = E.shape
    out = np.zeros((ny, nx))
    er = E / rho
    for j in range(ny):
        for i in range(nx + 1):
            f = fx[j, i]
            lo, hi = er[j, max(i - 1, 0)], er[j, min(i, nx - 1)]
            t = met.dSx[j, i] * f * (lo if f >= 0 else hi)
            if i > 0:
                out[j, i - 1] -= t
            if i < nx:
                out[j, i] += t
    for j in range(ny + 1):
        for i in range(nx):
            f = fy[j, i]
            lo, hi = er[max(j - 1, 0), i], er[min(j, ny - 1), i]
            t = met.dSy[j, i] * f * (lo if f >= 0 else hi)
            if j > 0:
                out[j - 1, i] -= t
            if j < ny:
                out[j, i] += t
    return out


@pytest.mark.parametrize("geom", [O.CARTESIAN, O.SPHERICAL])
def test_brute_force_and_conservation(geom):
    rng = np.random.default_rng(5)
    nx, ny = 7, 5
    if geom == O.CARTESIAN:
        xf, yf = np.cumsum(np.r_[0, rng.uniform(0.5, 1.5, nx)]), np.cumsum(np.r_[0, rng.uniform(0.5, 1.5, ny)])
    else:
        xf, yf = np.linspace(1.0, 3.0, nx + 1), np.linspace(0.2, 2.9, ny + 1)
    met = O.metrics(geom, xf, yf)
    E = 10 ** rng.uniform(0, 2, (ny, nx))
    rho = 10 ** rng.uniform(-1, 1, (ny, nx))
    fx, fy = rng.normal(size=(ny, nx + 1)), rng.normal(size=(ny + 1, nx))
    a = O.advection_volume_term(met, E, rho, fx, fy)
    np.testing.assert_allclose(a, brute_force(met, E, rho, fx, fy), rtol=1e-13, atol=1e-13 * np.abs(a).max())
    er = E / rho
    bnd = (np.sum(met.dSx[:, 0] * fx[:, 0] * er[:, 0]) - np.sum(met.dSx[:, -1] * fx[:, -1] * er[:, -1])
           + np.sum(met.dSy[0, :] * fy[0, :] * er[0, :]) - np.sum(met.dSy[-1, :] * fy[-1, :] * er[-1, :]))
    assert a.sum() == pytest.approx(bnd, rel=1e-12, abs=1e-12 * np.abs(a).max())


def test_uniform_er_in_divergence_free_flow():
    nx, ny = 6, 4
    met = O.metrics(O.CARTESIAN, np.linspace(0, 3, nx + 1), np.linspace(0, 2, ny + 1))
    rho = np.linspace(1.0, 2.0, nx * ny).reshape(ny, nx)
    E = 3.5 * rho
    fx = np.repeat(np.linspace(-1.0, 2.0, ny)[:, None], nx + 1, axis=1)  # constant along x
    fy = np.zeros((ny + 1, nx))
    a = O.advection_volume_term(met, E, rho, fx, fy)
    assert np.abs(a).max() <= 1e-14 * 3.5 * 2.0 * met.dSx.max()


def test_courant_one_shifts_by_one_cell():
    N, v, rho = 64, 2.0e4, 3.0
    xf = np.linspace(0.0, 1.0, N + 1)
    dx = xf[1] - xf[0]
    dt = dx / v
    E0 = 1.0 + np.exp(-((0.5 * (xf[1:] + xf[:-1]) - 0.3) / 0.05) ** 2)[None, :]
    E, T = E0.copy(), np.full((1, N), 10.0)
    fx, fy = np.full((1, N + 1), rho * v), np.zeros((2, N))
    one = np.ones((1, N))
    for k in range(1, 11):
        r = O.step(O.CARTESIAN, xf, np.array([0.0, 1.0]), E, T, rho * one, 1e30 * one, 0.0 * one, one, dt,
                   [O.BCSpec()] * 4, fx=fx, fy=fy)
        E, T = r.E, r.T
        expect = np.concatenate([np.full(k, E0[0, 0]), E0[0, :-k]])
        np.testing.assert_allclose(E[0], expect, rtol=1e-12)


def e4(N, t_end=6.2e-5):
    x0, x1, v, sig, E0 = -2.0, 14.0, 1.8e5, 1e7, 2e5
    xf = np.linspace(x0, x1, N + 1)
    dx = xf[1] - xf[0]
    xc = 0.5 * (xf[1:] + xf[:-1])
    E = np.where(np.abs(xc) < dx, E0 / (2 * dx), 1.0)[None, :]
    T = np.full((1, N), 0.1)
    dt = dx / v
    n = int(round(t_end / dt))
    one = np.ones((1, N))
    fx, fy = np.full((1, N + 1), v), np.zeros((2, N))  # rho = 1
    for _ in range(n):
        r = O.step(O.CARTESIAN, xf, np.array([0.0, 1.0]), E, T, one, sig * one, 0.0 * one, one, dt,
                   [O.BCSpec()] * 4, fx=fx, fy=fy)
        E, T = r.E, r.T
    t = n * dt
    D = O.C_LIGHT / (3 * sig)
    Ea = 1 + E0 / np.sqrt(4 * D * np.pi * t) * np.exp(-(xc - v * t) ** 2 / (4 * D * t))
    return E[0], Ea, dx, E0


def test_e4_moving_gaussian():
    errs = []
    for N in (512, 1024):
        E, Ea, dx, E0 = e4(N)
        errs.append(np.sum(np.abs(E - Ea)) / np.sum(Ea - 1))
        assert np.sum((E - 1) * dx) == pytest.approx(E0, rel=1e-6)
    packet = (Ea - 1) > 1e-3 * (Ea.max() - 1)
    assert np.max(np.abs(E - Ea)[packet] / Ea[packet]) < 0.05
    assert errs[1] < 1e-3
    assert errs[0] / errs[1] > 1.8, errs
