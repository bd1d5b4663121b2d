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


@pytest.mark.parametrize("prob", [W.make_c2(nx=13, ny=10), W.make_c5(nx=12, ny=10)], ids=lambda p: p.name)
def test_stop_rule_residuals_of_a_single_perturbation(prob):
    """The two stop-rule residuals (Section 3.2.1, ||b - A x|| < eps ||b||, in
    the per-volume and the Jacobi-scaled row forms) of the exact solution
    perturbed by delta in one cell c: the residual is then -delta times
    column c of M, i.e. -delta diag_c at c and +delta W at the faces c
    shares with its neighbours, written out here from the assembled
    coefficients cell by cell."""
    A = O.assemble_problem(prob)
    E = O.solve(A)
    ny, nx = A.diag.shape
    rhs = A.rhs
    for (j, i) in [(0, 0), (ny // 2, nx // 2), (ny - 1, nx - 1), (3, nx - 1)]:
        delta = 1e-3 * E[j, i]
        Ep = E.copy()
        Ep[j, i] += delta
        r = np.zeros((ny, nx))
        r[j, i] = -delta * A.diag[j, i]
        if i > 0:
            r[j, i - 1] += delta * A.W_x[j, i]
        if i + 1 < nx:
            r[j, i + 1] += delta * A.W_x[j, i + 1]
        if j > 0:
            r[j - 1, i] += delta * A.W_y[j, i]
        if j + 1 < ny:
            r[j + 1, i] += delta * A.W_y[j + 1, i]
        dV = A.met.dV
        row = np.sqrt(np.sum((r / dV) ** 2)) / np.sqrt(np.sum((rhs / dV) ** 2))
        s = 1.0 / np.sqrt(A.diag)
        scaled = np.sqrt(np.sum((s * r) ** 2)) / np.sqrt(np.sum((s * rhs) ** 2))
        # the unperturbed solution's own residual is rounding, far below these
        assert O.residual_rowform(A, Ep) == pytest.approx(row, rel=1e-6)
        assert O.residual_scaled(A, Ep) == pytest.approx(scaled, rel=1e-6)
    assert O.residual_scaled(A, E) < 1e-13
