"""Explicit radiation advection (Section 3.2.1 advection term) through the C
ABI (fld_set_mass_flux) against the oracle: random face mass fluxes on both
geometries, the paper's dynamical-diffusion test (moving Gaussian, 714 steps
replayed as one captured step graph) against the oracle and the analytic
solution, clearing the fluxes, and non-finite fluxes."""
import numpy as np
import pytest

import fld_workloads as W
from oracle import fld_oracle as O
from gpu_helpers import make_ctx, rel_l2, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def fluxes(prob, seed, scale):
    rng = np.random.default_rng(seed)
    ny, nx = prob.E.shape
    return scale * rng.normal(size=(ny, nx + 1)), scale * rng.normal(size=(ny + 1, nx))


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("name,kw,prec,norm", [
    ("c1", dict(nx=48, ny=40), "mixed", 0),
    ("c5", dict(nx=64, ny=48), "fp64", 1),
])
def test_advection_step_matches_oracle(lib, name, kw, prec, norm):
    prob = W.make(name, **kw)
    # fluxes sized so that dt S_adv is a sizeable part of E (|f| dt dS / dV ~ 0.1 rho)
    met = O.metrics(prob.geom, prob.x_faces, prob.y_faces)
    scale = 0.1 * float(np.median(prob.rho)) * float(np.median(met.dV / met.dSx[:, :-1])) / prob.dt
    fx, fy = fluxes(prob, 3, scale)
    ref = O.step_problem(prob, fx=fx, fy=fy)
    assert rel_l2(ref.E, O.step_problem(prob).E) > 1e-6  # the term moves E far beyond the tolerance
    ctx = make_ctx(lib, prob, precision=prec, norm=norm, rel_tol=1e-12)
    t = to_dev(prob, torch)
    dfx, dfy = dev(fx), dev(fy)
    ctx.set_mass_flux(dfx, dfy)
    info = ctx.step(t["E"], t["T"], t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], prob.dt, t["ghost_E"],
                    check=False)
    torch.cuda.synchronize()
    assert info["status"] == 0
    assert rel_l2(t["E"].cpu().numpy(), ref.E) < 1e-10 and rel_l2(t["T"].cpu().numpy(), ref.T) < 1e-10
    # clearing the fluxes gives the plain step bit for bit
    ctx.set_mass_flux(None, None)
    t2 = to_dev(prob, torch)
    ctx.step(t2["E"], t2["T"], t2["rho"], t2["kappa_R"], t2["kappa_P"], t2["c_v"], prob.dt, t2["ghost_E"], check=False)
    ctx.close()
    ctx = make_ctx(lib, prob, precision=prec, norm=norm, rel_tol=1e-12)
    t3 = to_dev(prob, torch)
    ctx.step(t3["E"], t3["T"], t3["rho"], t3["kappa_R"], t3["kappa_P"], t3["c_v"], prob.dt, t3["ghost_E"], check=False)
    torch.cuda.synchronize()
    assert np.array_equal(t2["E"].cpu().numpy(), t3["E"].cpu().numpy())
    ctx.close()


def e4_problem(N=1024):
    x0, x1, v, sig, E0 = -2.0, 14.0, 1.8e5, 1e7, 2e5
    xf = np.linspace(x0, x1, N + 1)
    dx = xf[1] - xf[0]
    xc = 0.5 * (xf[1:] + xf[:-1])
    one = np.ones((1, N))
    prob = W.Problem("e4", W.GEOM_CARTESIAN, xf, np.array([0.0, 1.0]),
                     np.where(np.abs(xc) < dx, E0 / (2 * dx), 1.0)[None, :], 0.1 * one, one.copy(), sig * one,
                     0.0 * one, one.copy(), dx / v, [W.BC()] * 4)
    return prob, xc, v, sig, E0


def test_e4_moving_gaussian_on_gpu(lib):
    prob, xc, v, sig, E0 = e4_problem()
    n = int(round(6.2e-5 / prob.dt))
    fx, fy = np.full((1, prob.nx + 1), v), np.zeros((2, prob.nx))
    # oracle: the same n steps
    E, T = prob.E, prob.T
    for _ in range(n):
        r = O.step_problem(prob, E, T, fx=fx, fy=fy)
        E, T = r.E, r.T
    ctx = make_ctx(lib, prob, precision="mixed", norm=1, rel_tol=1e-12)
    t = to_dev(prob, torch)
    ctx.set_mass_flux(dev(fx), dev(fy))
    infos = ctx.steps(n, t["E"], t["T"], t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], prob.dt, check=False)
    torch.cuda.synchronize()
    ctx.close()
    assert all(i["status"] == 0 for i in infos)
    Eg = t["E"].cpu().numpy()
    assert rel_l2(Eg, E) < 1e-9
    tt = n * prob.dt
    D = O.C_LIGHT / (3 * sig)
    Ea = 1 + E0 / np.sqrt(4 * D * np.pi * tt) * np.exp(-(xc - v * tt) ** 2 / (4 * D * tt))
    assert np.sum(np.abs(Eg[0] - Ea)) / np.sum(Ea - 1) < 1e-3


def test_nonfinite_flux_is_reported(lib):
    prob = W.make("c1", nx=24, ny=20)
    fx, fy = fluxes(prob, 4, 1.0)
    fx[3, 5] = np.nan
    ctx = make_ctx(lib, prob)
    t = to_dev(prob, torch)
    ctx.set_mass_flux(dev(fx), dev(fy))
    info = ctx.step(t["E"], t["T"], t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], prob.dt, t["ghost_E"],
                    check=False)
    assert info["status"] == lib.FLD_ENONFINITE
    ctx.close()
