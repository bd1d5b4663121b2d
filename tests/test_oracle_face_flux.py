"""Pins for the face-flux export (Section 3.2.1 flux formula).

* Without gas coupling a step is a discrete conservation law: every cell
  satisfies dV (E^{n+1} - E^n) = -dt (sum of its faces' outward F dS), with
  the fluxes of every boundary kind (both geometries, random grids).
* Interior fluxes equal -D (E_hi - E_lo) / h with the assembled D.
* The steady slab (inward flux F against a Milne side) carries F through
  every face.
"""
import numpy as np
import pytest

from oracle import fld_oracle as O


def random_case(geom, kinds, seed):
    rng = np.random.default_rng(seed)
    nx, ny = 9, 7
    if geom == O.CARTESIAN:
        xf = np.cumsum(np.r_[0.0, rng.uniform(0.5, 1.5, nx)])
        yf = np.cumsum(np.r_[0.0, rng.uniform(0.5, 1.5, ny)])
    else:
        xf = np.linspace(1.0, 3.0, nx + 1)
        yf = np.linspace(0.0, np.pi, ny + 1)
    shp = (ny, nx)
    T = 10 ** rng.uniform(3, 4, shp)
    E = O.A_RAD * T ** 4 * 10 ** rng.uniform(-0.5, 0.5, shp)
    rho = 10 ** rng.uniform(-1, 0, shp)
    kR = 10 ** rng.uniform(-1, 1, shp)
    bcs = []
    for s, k in enumerate(kinds):
        n = ny if s < 2 else nx
        g = O.A_RAD * (10 ** rng.uniform(3, 4, n)) ** 4 if k == O.DIRICHLET_GHOST else None
        v = {O.DIRICHLET_FACE: 5e3, O.FLUX_IN: 1e9}.get(k, 0.0)
        bcs.append(O.BCSpec(k, v, g))
    return xf, yf, E, T, rho, kR, bcs


@pytest.mark.parametrize("geom,kinds", [
    (O.CARTESIAN, [O.DIRICHLET_FACE, O.FREE_STREAM, O.FLUX_IN, O.MILNE]),
    (O.CARTESIAN, [O.DIRICHLET_GHOST, O.MILNE, O.REFLECT, O.DIRICHLET_GHOST]),
    (O.SPHERICAL, [O.FLUX_IN, O.MILNE, O.AXIS, O.AXIS]),
    (O.SPHERICAL, [O.DIRICHLET_FACE, O.FREE_STREAM, O.AXIS, O.AXIS]),
])
def test_conservation_without_coupling(geom, kinds):
    xf, yf, E, T, rho, kR, bcs = random_case(geom, kinds, 4)
    dt = 3e-11
    zero = np.zeros_like(E)
    r = O.step(geom, xf, yf, E, T, rho, kR, zero, np.ones_like(E), dt, bcs, O.LIMITER_LP)
    Fx, Fy = O.face_fluxes(r.A, E, r.E, kR * rho, dt, bcs, O.LIMITER_LP)
    met = r.A.met
    out = (Fx[:, 1:] * met.dSx[:, 1:] - Fx[:, :-1] * met.dSx[:, :-1]
           + Fy[1:, :] * met.dSy[1:, :] - Fy[:-1, :] * met.dSy[:-1, :])
    lhs = met.dV * (r.E - E)
    np.testing.assert_allclose(lhs, -dt * out, rtol=1e-8, atol=1e-10 * np.abs(lhs).max())
    # interior faces: -D grad E with the assembled D
    np.testing.assert_allclose(Fx[:, 1:-1], O.interface_flux_x(r.A, r.E), rtol=1e-12,
                               atol=1e-14 * np.abs(Fx).max())


def test_steady_slab_carries_the_inflow():
    N, F, sig = 50, 4.0e12, 3.0
    xf = np.linspace(0.0, 2.0, N + 1)
    one = np.ones((1, N))
    bcs = [O.BCSpec(O.FLUX_IN, F), O.BCSpec(O.MILNE), O.BCSpec(), O.BCSpec()]
    E0 = 1e3 * one
    r = O.step(O.CARTESIAN, xf, np.array([0.0, 1.0]), E0, 1e3 * one, one, sig * one, 0.0 * one, one, 1e6, bcs)
    Fx, Fy = O.face_fluxes(r.A, E0, r.E, sig * one, 1e6, bcs)
    np.testing.assert_allclose(Fx[0], F, rtol=1e-8)
    assert np.all(Fy == 0.0)
