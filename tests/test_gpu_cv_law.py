"""Temperature-dependent heat capacity (Section 3.2.1, the C_V step that the
radiation-subsystem algorithm repeats before every sub-step; Section 5.1.2,
a nonlinear gas energy linearised with C_V = de_g/dT) through the C ABI
(fld_set_cv_law) against the oracle's sub-cycled step with the same power law
c_v(T) = c_v,ref (T / T_ref)^p: geometric and coupling-limited sub-steps,
multi-step graph replays (the law's kernel captured with the step), the
cooling 0D coupling set-up of Section 5.1.1 where the law changes the answer,
p = 0 restoring the fixed c_v, and the argument checks."""
import numpy as np
import pytest

import fld_workloads as W
from oracle import fld_oracle as O
from oracle import fld_substep as S
from gpu_helpers import make_ctx, rel_l2, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

K_B = 1.380649e-16
M_H = 1.6735575e-24


def perturbed(name, seed=11, **kw):
    prob = W.make(name, **kw)
    rng = np.random.default_rng(seed)
    prob.T = prob.T * (1.0 + 0.3 * rng.uniform(-1.0, 1.0, prob.T.shape))
    return prob


def run_gpu(fld, prob, law, sub=None, nsteps=None, **opt):
    ctx = make_ctx(fld, prob, **opt)
    if law is not None:
        ctx.set_cv_law(*law)
    t = to_dev(prob, torch)
    args = (t["E"], t["T"], t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"])
    if nsteps is None:
        r = ctx.substep(*args, prob.dt, ghost_E=t["ghost_E"], check=False, **sub)
    else:
        infos = ctx.steps(nsteps, *args, prob.dt, ghost_E=t["ghost_E"], check=False)
        r = dict(status=max(i["status"] for i in infos), infos=infos)
    torch.cuda.synchronize()
    out = t["E"].cpu().numpy(), t["T"].cpu().numpy(), r
    ctx.close()
    return out


@pytest.mark.parametrize("name,kw,prec,norm,p", [
    ("c1", dict(nx=48, ny=40), "mixed", 0, 1.5),
    ("c5", dict(nx=64, ny=48), "fp64", 1, -0.7),
])
def test_geometric_substeps_with_law_match_oracle(lib, name, kw, prec, norm, p):
    prob = perturbed(name, **kw)
    law = (float(np.mean(prob.T)), p)
    E, T, r = run_gpu(lib, prob, law, dict(n_sub=4, q=1.5), precision=prec, norm=norm, rel_tol=1e-12)
    assert r["status"] == 0 and all(i["status"] == 0 for i in r["infos"])
    ref = S.substep_problem(prob, n_sub=4, q=1.5, cv_law=law)
    fixed = S.substep_problem(prob, n_sub=4, q=1.5)
    print(name, prec, rel_l2(T, ref.T), "law vs fixed", rel_l2(ref.T, fixed.T), flush=True)
    assert rel_l2(T, fixed.T) > 1e-6  # the law changes the answer
    assert rel_l2(E, ref.E) < 1e-10 and rel_l2(T, ref.T) < 1e-10


def test_multistep_graph_with_law_matches_oracle(lib):
    prob = perturbed("c1", nx=40, ny=36)
    law = (float(np.mean(prob.T)), 1.5)
    E, T, r = run_gpu(lib, prob, law, nsteps=6, precision="mixed", rel_tol=1e-12)
    assert r["status"] == 0
    bcs = O.bcs_from_problem(prob)
    Er, Tr = prob.E, prob.T
    for _ in range(6):
        s = S.substep(prob.geom, prob.x_faces, prob.y_faces, Er, Tr, prob.rho, prob.kappa_R, prob.kappa_P,
                      prob.c_v, prob.dt, bcs, n_sub=1, cv_law=law)
        Er, Tr = s.E, s.T
    assert rel_l2(E, Er) < 1e-10 and rel_l2(T, Tr) < 1e-10


def test_e1_cooling_coupling_limited_with_law(lib):
    """Cooling gas (e_g = 1e10 erg/cm^3) on the Section 5.1.1 set-up with
    c_v growing as T^1.5 about the radiation temperature."""
    rho, kP, mu, nx = 1e-7, 0.4, 0.6, 16
    cv = 3.0 * K_B / (2.0 * mu * M_H)
    shape = (1, nx)
    prob = W.Problem("e1", W.GEOM_CARTESIAN, np.linspace(0.0, 1.0, nx + 1), np.linspace(0.0, 1.0, 2),
                     np.full(shape, 1e12), np.full(shape, 1e10 / (rho * cv)), np.full(shape, rho),
                     np.full(shape, 1e10 / rho), np.full(shape, kP), np.full(shape, cv), 3e-7, [W.BC()] * 4)
    law = ((1e12 / O.A_RAD) ** 0.25, 1.5)
    E, T, r = run_gpu(lib, prob, law, dict(dbar=0.04, max_sub=1000), precision="fp64", norm=1, rel_tol=1e-12)
    ref = S.substep_problem(prob, dbar=0.04, max_sub=1000, cv_law=law)
    fixed = S.substep_problem(prob, dbar=0.04, max_sub=1000)
    assert r["status"] == 0 and len(r["dts"]) == len(ref.dts) > 100
    assert len(ref.dts) != len(fixed.dts)
    np.testing.assert_allclose(r["dts"], ref.dts, rtol=1e-8)
    np.testing.assert_allclose(T, ref.T, rtol=1e-9)
    np.testing.assert_allclose(E, ref.E, rtol=1e-9)


def test_p0_restores_fixed_cv_and_errors(lib):
    prob = perturbed("c1", nx=32, ny=30)
    E0, T0, _ = run_gpu(lib, prob, None, dict(n_sub=3, q=1.3))
    ctx = make_ctx(lib, prob)
    for bad in ((0.0, 1.0), (-1.0, 1.0), (float("nan"), 1.0), (1.0, float("inf"))):
        with pytest.raises(lib.FLDError) as e:
            ctx.set_cv_law(*bad)
        assert e.value.status == lib.FLD_EINVAL
    ctx.set_cv_law(float(np.mean(prob.T)), 2.0)
    ctx.set_cv_law(5.0, 0.0)
    t = to_dev(prob, torch)
    r = ctx.substep(t["E"], t["T"], t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], prob.dt, ghost_E=t["ghost_E"],
                    n_sub=3, q=1.3, check=False)
    torch.cuda.synchronize()
    assert r["status"] == 0
    assert np.array_equal(t["E"].cpu().numpy(), E0) and np.array_equal(t["T"].cpu().numpy(), T0)
    ctx.close()
