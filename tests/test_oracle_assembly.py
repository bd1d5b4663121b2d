"""Pins for the oracle's assembled system (Section 3.2.1 coefficients, Section 2 physics).

* symmetry and strict diagonal dominance of the volume-weighted E system;
* equilibrium: T_g = T_rad uniform stays fixed for any rho / kappa fields;
* energy conservation: the change of sum dV (E + C_V T) equals the energy
  that crossed the boundary faces, for every boundary kind and geometry.
"""
import numpy as np
import pytest

from oracle import fld_oracle as O
import fld_workloads as W


def small_problems():
    yield W.make_c1(nx=12, ny=9)
    yield W.make_c2(nx=13, ny=10)
    yield W.make_c3(nx=14, ny=8)
    yield W.make_c5(nx=12, ny=10)
    yield W.make_c4_block(3, 16, 12)


@pytest.mark.parametrize("prob", list(small_problems()), ids=lambda p: p.name)
def test_symmetric_and_diagonally_dominant(prob):
    A = O.assemble_problem(prob)
    M = A.M.toarray()
    assert np.array_equal(M, M.T)
    off = np.abs(M).sum(axis=1) - np.abs(np.diag(M))
    mass = (A.met.dV * (1.0 + A.beta * A.f)).ravel()
    assert np.all(np.diag(M) - off >= mass * (1 - 1e-12) - 1e-14 * off)
    assert np.all(mass > 0)
    np.linalg.cholesky(M / np.sqrt(np.outer(np.diag(M), np.diag(M))))


def equilibrium_case(prob, Tval):
    T0 = np.full(prob.T.shape, Tval)
    E0 = O.A_RAD * T0 ** 4
    bcs = O.bcs_from_problem(prob)
    for b in bcs:
        if b.kind == O.DIRICHLET_FACE:
            b.value = Tval
        elif b.kind == O.DIRICHLET_GHOST:
            b.ghost = np.full_like(b.ghost, O.A_RAD * Tval ** 4)
        elif b.kind in (O.FLUX_IN, O.FREE_STREAM):
            b.kind = O.REFLECT
    return T0, E0, bcs


@pytest.mark.parametrize("prob", list(small_problems()), ids=lambda p: p.name)
def test_equilibrium_is_fixed_point(prob):
    T0, E0, bcs = equilibrium_case(prob, 6.5e3)
    A = O.assemble(prob.geom, prob.x_faces, prob.y_faces, E0, T0, prob.rho, prob.kappa_R,
                   prob.kappa_P, prob.c_v, prob.dt, bcs)
    # the equilibrium state satisfies the assembled rows to rounding
    r = A.rhs.ravel() - A.M @ E0.ravel()
    scale = np.abs(A.diag.ravel() * E0.ravel()) + np.abs(A.rhs.ravel())
    assert np.max(np.abs(r) / scale) < 1e-14
    # the gas update leaves T fixed when E^{n+1} = a_R T^4
    np.testing.assert_allclose(O.gas_update(A, T0, E0), T0, rtol=1e-14)
    # and the full step returns it (up to the direct solve's conditioning)
    E1 = O.solve(A)
    np.testing.assert_allclose(E1, E0, rtol=1e-9)


@pytest.mark.parametrize("prob", list(small_problems()), ids=lambda p: p.name)
def test_energy_conservation(prob):
    res = O.step_problem(prob)
    A = res.A
    before = O.total_energy(A, prob.E, prob.T)
    after = O.total_energy(A, res.E, res.T)
    inflow = O.boundary_energy_input(prob.geom, A, O.bcs_from_problem(prob), res.E, prob.dt)
    # the iterative / rounding discrepancy is bounded by sum dV r_hat; direct solve: tiny
    scale = max(abs(before), abs(after))
    assert abs((after - before) - inflow) <= 1e-11 * scale


def test_conservation_all_boundary_kinds_cartesian():
    prob = W.make_c2(nx=9, ny=7)
    rng = np.random.default_rng(11)
    ghost = O.A_RAD * rng.uniform(3e3, 9e3, 7) ** 4
    bcs = [O.BCSpec(O.DIRICHLET_FACE, 1.5e4), O.BCSpec(O.DIRICHLET_GHOST, 0.0, ghost),
           O.BCSpec(O.FLUX_IN, 3e12), O.BCSpec(O.FREE_STREAM)]
    res = O.step(prob.geom, prob.x_faces, prob.y_faces, prob.E, prob.T, prob.rho, prob.kappa_R,
                 prob.kappa_P, prob.c_v, prob.dt, bcs)
    d = O.total_energy(res.A, res.E, res.T) - O.total_energy(res.A, prob.E, prob.T)
    inflow = O.boundary_energy_input(prob.geom, res.A, bcs, res.E, prob.dt)
    assert inflow != 0.0
    assert abs(d - inflow) <= 1e-11 * abs(O.total_energy(res.A, prob.E, prob.T))
