"""Brute-force pins (Section 3.2.1 linear system).

The oracle's reduced solve (T eliminated, volume-weighted, sparse LU) is
checked against the paper's coupled 2 N1 N2 system written literally from the
phi/psi coefficient list (oracle/coupled.py, pure-Python loops):

* the oracle's (E^{n+1}, T^{n+1}) satisfy every phi and psi row to rounding;
* a dense LAPACK solve of the coupled system agrees (it loses a few digits
  to the rows' scaling, hence the looser bound);
* the reduced matrix equals a dense LAPACK solve of itself on tiny grids;

on fixed cases and on random grids of 2..8 x 2..8 cells, both geometries,
every boundary kind (hypothesis).
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

from oracle import fld_oracle as O
from oracle.coupled import coupled_system, solve_coupled


def random_case(rng, nx, ny, geom, kinds):
    if geom == O.CARTESIAN:
        xf = np.concatenate([[0.0], np.cumsum(rng.uniform(0.5, 2.0, nx))]) * 1e10
        yf = np.concatenate([[0.0], np.cumsum(rng.uniform(0.5, 2.0, ny))]) * 1e10
    else:
        xf = np.exp(np.linspace(np.log(1e11), np.log(1e11 * rng.uniform(2, 50)), nx + 1))
        yf = np.linspace(0.0, np.pi, ny + 1)
    shape = (ny, nx)
    T = rng.uniform(2e3, 3e4, shape)
    E = O.A_RAD * (T * rng.uniform(0.7, 1.3, shape)) ** 4
    rho = 10 ** rng.uniform(-12, -7, shape)
    kR = 10 ** rng.uniform(-3, 3, shape)
    kP = 10 ** rng.uniform(-3, 3, shape)
    cv = 10 ** rng.uniform(6, 9, shape)
    dt = 10 ** rng.uniform(0, 4)
    bcs = []
    for s, k in enumerate(kinds):
        n = ny if s < 2 else nx
        if k == O.DIRICHLET_FACE:
            bcs.append(O.BCSpec(k, rng.uniform(3e3, 3e4)))
        elif k == O.DIRICHLET_GHOST:
            bcs.append(O.BCSpec(k, 0.0, O.A_RAD * rng.uniform(3e3, 3e4, n) ** 4))
        elif k == O.FLUX_IN:
            bcs.append(O.BCSpec(k, 10 ** rng.uniform(8, 13)))
        else:
            bcs.append(O.BCSpec(k))
    return xf, yf, E, T, rho, kR, kP, cv, dt, bcs


def check_case(case, limiter=O.LIMITER_LP):
    xf, yf, E, T, rho, kR, kP, cv, dt, bcs = case
    geom = O.SPHERICAL if xf[0] > 0 and yf[-1] == np.pi else O.CARTESIAN
    res = O.step(geom, xf, yf, E, T, rho, kR, kP, cv, dt, bcs, limiter)
    A = res.A
    Amat, b = coupled_system(A, E, T, rho, kP, cv, dt)
    x = np.empty(b.size)
    x[0::2] = res.E.ravel()
    x[1::2] = res.T.ravel()
    r = b - Amat @ x
    scale = np.abs(Amat) @ np.abs(x) + np.abs(b)
    assert np.max(np.abs(r) / scale) < 1e-12
    Ec, Tc = solve_coupled(A, E, T, rho, kP, cv, dt)
    # LAPACK on the unscaled coupled rows loses digits to their conditioning
    assert np.linalg.norm(res.E - Ec) <= 1e-6 * np.linalg.norm(res.E)
    assert np.linalg.norm(res.T - Tc) <= 1e-6 * np.linalg.norm(res.T)
    Md = A.M.toarray()
    Ed = np.linalg.solve(Md, A.rhs.ravel()).reshape(res.E.shape)
    np.testing.assert_allclose(res.E, Ed, rtol=1e-8)


@pytest.mark.parametrize("geom", [O.CARTESIAN, O.SPHERICAL])
@pytest.mark.parametrize("limiter", [O.LIMITER_LP, O.LIMITER_MINERBO, O.LIMITER_DIFFUSION])
def test_fixed_cases(geom, limiter):
    rng = np.random.default_rng(100 + geom * 10 + limiter)
    if geom == O.CARTESIAN:
        kinds = [O.DIRICHLET_FACE, O.FREE_STREAM, O.DIRICHLET_GHOST, O.FLUX_IN]
    else:
        kinds = [O.FLUX_IN, O.FREE_STREAM, O.AXIS, O.AXIS]
    check_case(random_case(rng, 6, 5, geom, kinds), limiter)


CART_KINDS = [O.REFLECT, O.DIRICHLET_FACE, O.DIRICHLET_GHOST, O.FLUX_IN, O.FREE_STREAM]


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(nx=st.integers(1, 8), ny=st.integers(1, 8), seed=st.integers(0, 2 ** 31),
       geom=st.sampled_from([O.CARTESIAN, O.SPHERICAL]),
       kinds=st.lists(st.sampled_from(CART_KINDS), min_size=4, max_size=4))
def test_random_grids(nx, ny, seed, geom, kinds):
    rng = np.random.default_rng(seed)
    if geom == O.SPHERICAL:
        kinds = kinds[:2] + [O.AXIS, O.AXIS]
        kinds = [k if k != O.DIRICHLET_GHOST else O.REFLECT for k in kinds]
    check_case(random_case(rng, nx, ny, geom, kinds))
