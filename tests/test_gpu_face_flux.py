"""Face-flux export (Section 3.2.1 flux formula) through the C ABI
(fld_face_flux, and fld_substep's sub-step average) against the oracle's
face fluxes, with every boundary kind on both geometries, and the discrete
balance of a step without gas coupling on the GPU's own fields."""
import numpy as np
import pytest

import fld_workloads as W
from oracle import fld_oracle as O
from oracle import fld_substep as S
from gpu_helpers import make_ctx, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def case(name):
    if name == "cart":
        prob = W.make("c1", nx=48, ny=40)
        prob.bc = [W.BC(W.BC_DIRICHLET_FACE, 2.0e4), W.BC(W.BC_FREE_STREAM), W.BC(W.BC_FLUX_IN, 1.0e12),
                   W.BC(W.BC_MILNE)]
        prob.ghost_E = None
    else:
        prob = W.make("c5", nx=64, ny=48)
        prob.bc[1] = W.BC(W.BC_MILNE)
    return prob


def run_step(lib, prob, prec):
    ctx = make_ctx(lib, prob, precision=prec, rel_tol=1e-12, norm=1)
    t = to_dev(prob, torch)
    info = ctx.step(t["E"], t["T"], t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], prob.dt, t["ghost_E"],
                    check=False)
    ny, nx = prob.E.shape
    Fx = torch.zeros((ny, nx + 1), dtype=torch.float64, device="cuda")
    Fy = torch.zeros((ny + 1, nx), dtype=torch.float64, device="cuda")
    ctx.face_flux(t["E"], Fx, Fy)
    torch.cuda.synchronize()
    ctx.close()
    return info, t["E"].cpu().numpy(), Fx.cpu().numpy(), Fy.cpu().numpy()


@pytest.mark.parametrize("name,prec", [("cart", "mixed"), ("cart", "fp64"), ("sph", "fp64")])
def test_face_flux_matches_oracle(lib, name, prec):
    prob = case(name)
    info, E, Fx, Fy = run_step(lib, prob, prec)
    assert info["status"] == 0
    ref = O.step_problem(prob)
    bcs = O.bcs_from_problem(prob)
    Rx, Ry = O.face_fluxes(ref.A, prob.E, ref.E, prob.kappa_R * prob.rho, prob.dt, bcs)
    scale = max(np.abs(Rx).max(), np.abs(Ry).max())
    np.testing.assert_allclose(Fx, Rx, rtol=1e-7, atol=1e-8 * scale)
    np.testing.assert_allclose(Fy, Ry, rtol=1e-7, atol=1e-8 * scale)


def test_balance_without_coupling(lib):
    prob = case("cart")
    prob.kappa_P = np.zeros_like(prob.kappa_P)
    info, E, Fx, Fy = run_step(lib, prob, "fp64")
    met = O.metrics(prob.geom, prob.x_faces, prob.y_faces)
    out = (Fx[:, 1:] * met.dSx[:, 1:] - Fx[:, :-1] * met.dSx[:, :-1]
           + Fy[1:, :] * met.dSy[1:, :] - Fy[:-1, :] * met.dSy[:-1, :])
    lhs = met.dV * (E - prob.E)
    np.testing.assert_allclose(lhs, -prob.dt * out, rtol=1e-6, atol=1e-9 * np.abs(lhs).max())


def test_substep_average(lib):
    prob = case("cart")
    ctx = make_ctx(lib, prob, precision="fp64", rel_tol=1e-12, norm=1)
    t = to_dev(prob, torch)
    ny, nx = prob.E.shape
    Fx = torch.zeros((ny, nx + 1), dtype=torch.float64, device="cuda")
    Fy = torch.zeros((ny + 1, nx), dtype=torch.float64, device="cuda")
    r = ctx.substep(t["E"], t["T"], t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], prob.dt, n_sub=3, q=1.5,
                    check=False, Fx=Fx, Fy=Fy)
    torch.cuda.synchronize()
    ctx.close()
    assert r["status"] == 0
    ref = S.substep_problem(prob, n_sub=3, q=1.5)
    ax, ay = ref.Fx, ref.Fy
    scale = max(np.abs(ax).max(), np.abs(ay).max())
    np.testing.assert_allclose(Fx.cpu().numpy(), ax, rtol=1e-7, atol=1e-8 * scale)
    np.testing.assert_allclose(Fy.cpu().numpy(), ay, rtol=1e-7, atol=1e-8 * scale)


def test_face_flux_needs_a_step(lib):
    prob = case("cart")
    ctx = make_ctx(lib, prob)
    t = to_dev(prob, torch)
    with pytest.raises(lib.FLDError):
        ctx.face_flux(t["E"], torch.zeros((prob.ny, prob.nx + 1), dtype=torch.float64, device="cuda"))
    ctx.close()


def test_advection_substeps_and_fluxes_together(lib):
    """Advection, sub-cycling and the sub-step-averaged face fluxes at once,
    against the oracle's sub-cycled steps with the same mass fluxes."""
    prob = case("cart")
    rng = np.random.default_rng(9)
    ny, nx = prob.E.shape
    met = O.metrics(prob.geom, prob.x_faces, prob.y_faces)
    scale = 0.05 * float(np.median(prob.rho)) * float(np.median(met.dV / met.dSx[:, :-1])) / prob.dt
    fx, fy = scale * rng.normal(size=(ny, nx + 1)), scale * rng.normal(size=(ny + 1, nx))
    ctx = make_ctx(lib, prob, precision="fp64", rel_tol=1e-12, norm=1)
    t = to_dev(prob, torch)
    dfx = torch.tensor(fx, dtype=torch.float64, device="cuda")
    dfy = torch.tensor(fy, dtype=torch.float64, device="cuda")
    ctx.set_mass_flux(dfx, dfy)
    Fx = torch.zeros((ny, nx + 1), dtype=torch.float64, device="cuda")
    Fy = torch.zeros((ny + 1, nx), dtype=torch.float64, device="cuda")
    r = ctx.substep(t["E"], t["T"], t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], prob.dt, n_sub=3, q=1.4,
                    check=False, Fx=Fx, Fy=Fy)
    torch.cuda.synchronize()
    ctx.close()
    assert r["status"] == 0
    bcs = O.bcs_from_problem(prob)
    ref = S.substep(prob.geom, prob.x_faces, prob.y_faces, prob.E, prob.T, prob.rho, prob.kappa_R, prob.kappa_P,
                    prob.c_v, prob.dt, bcs, n_sub=3, q=1.4, fx=fx, fy=fy)
    from gpu_helpers import rel_l2
    assert rel_l2(t["E"].cpu().numpy(), ref.E) < 1e-10 and rel_l2(t["T"].cpu().numpy(), ref.T) < 1e-10
    ax, ay = ref.Fx, ref.Fy
    sc = max(np.abs(ax).max(), np.abs(ay).max())
    np.testing.assert_allclose(Fx.cpu().numpy(), ax, rtol=1e-7, atol=1e-8 * sc)
    np.testing.assert_allclose(Fy.cpu().numpy(), ay, rtol=1e-7, atol=1e-8 * sc)


def test_substep_balance_on_gpu_fields(lib):
    """The GPU's own sub-cycled step closes every cell's energy balance with
    its averaged fluxes and the step-start advection term (Section 3.2.1 flux
    formula with D^n outside the sub-step sum):
    dV (E^end - E^n) + dV C_V (T^end - T^n) = -dt sum_faces F dS + dt dV S_adv(E^n)."""
    prob = case("cart")
    rng = np.random.default_rng(5)
    ny, nx = prob.E.shape
    prob.T = prob.T * (1.0 + 0.3 * rng.uniform(-1.0, 1.0, prob.T.shape))
    met = O.metrics(prob.geom, prob.x_faces, prob.y_faces)
    scale = 0.05 * float(np.median(prob.rho)) * float(np.median(met.dV / met.dSx[:, :-1])) / prob.dt
    fx, fy = scale * rng.normal(size=(ny, nx + 1)), scale * rng.normal(size=(ny + 1, nx))
    ctx = make_ctx(lib, prob, precision="fp64", rel_tol=1e-12, norm=1)
    t = to_dev(prob, torch)
    ctx.set_mass_flux(torch.tensor(fx, dtype=torch.float64, device="cuda"),
                      torch.tensor(fy, dtype=torch.float64, device="cuda"))
    Fx = torch.zeros((ny, nx + 1), dtype=torch.float64, device="cuda")
    Fy = torch.zeros((ny + 1, nx), dtype=torch.float64, device="cuda")
    r = ctx.substep(t["E"], t["T"], t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], prob.dt, n_sub=4, q=1.6,
                    check=False, Fx=Fx, Fy=Fy)
    torch.cuda.synchronize()
    ctx.close()
    assert r["status"] == 0
    E, T, Fx, Fy = t["E"].cpu().numpy(), t["T"].cpu().numpy(), Fx.cpu().numpy(), Fy.cpu().numpy()
    out = (Fx[:, 1:] * met.dSx[:, 1:] - Fx[:, :-1] * met.dSx[:, :-1]
           + Fy[1:, :] * met.dSy[1:, :] - Fy[:-1, :] * met.dSy[:-1, :])
    adv = O.advection_volume_term(met, prob.E, prob.rho, fx, fy)
    CV = prob.rho * prob.c_v
    lhs = met.dV * (E - prob.E) + met.dV * CV * (T - prob.T)
    rhs = -prob.dt * out + prob.dt * adv
    big = np.abs(met.dV * (E - prob.E)).max() + np.abs(prob.dt * adv).max() + np.abs(prob.dt * out).max()
    # the solves stop at a 1e-12 scaled residual: that, not rounding, bounds the balance
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-8 * big)
