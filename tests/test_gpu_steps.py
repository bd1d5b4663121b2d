"""Multi-step runs (Section 3.2.1 sub-step loop): fld_steps (steps queued back
to back, iterations in captured chunks read ahead by the host) and
fld_steps_graph (steps after the first replay one captured hipGraph), against
repeated fld_step calls (bit-identical) and against the FP64 oracle stepped
the same number of times."""
import numpy as np
import pytest

import fld_workloads as W
from oracle import fld_oracle as O
from gpu_helpers import make_ctx, rel_l2, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _run(fld, torch, prob, nsteps, multi, profile=False, **opt):
    ctx = make_ctx(fld, prob, **opt)
    t = to_dev(prob, torch)
    args = (t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], prob.dt, t["ghost_E"])
    if profile:
        ctx.profile(True)
    if multi == "graph":
        infos = ctx.steps_graph(nsteps, t["E"], t["T"], *args, check=False)
    elif multi:
        infos = ctx.steps(nsteps, t["E"], t["T"], *args, check=False)
    else:
        infos = [ctx.step(t["E"], t["T"], *args, check=False) for _ in range(nsteps)]
    torch.cuda.synchronize()
    out = t["E"].cpu().numpy(), t["T"].cpu().numpy(), infos
    ctx.close()
    return out


def _oracle_steps(prob, nsteps):
    E, T = prob.E, prob.T
    for _ in range(nsteps):
        r = O.step_problem(prob, E, T)
        E, T = r.E, r.T
    return E, T


@pytest.mark.parametrize("mode", ["steps", "graph"])
@pytest.mark.parametrize("name,kw,prec,norm,cyc,cm", [
    ("c1", dict(nx=48, ny=40), "mixed", 0, 1, 256),
    ("c2", dict(nx=70, ny=52), "fp64", 0, 1, 256),
    ("c5", dict(nx=96, ny=64), "mixed", 1, 1, 256),
    ("c5", dict(nx=512, ny=256), "mixed", 1, 4, 256),
    ("c5", dict(nx=512, ny=256), "fp64", 1, 3, 256),
    ("c5", dict(nx=512, ny=256), "mixed", 1, 4, 2048),
    ("c5", dict(nx=512, ny=256), "fp64", 1, 3, 2048),
])
def test_steps_equal_repeated_step(lib, name, kw, prec, norm, cyc, cm, mode):
    fld = lib
    prob = W.make(name, **kw)
    print(f"[steps] {name} {prob.nx}x{prob.ny} {prec} cycle {cyc} coarse {cm} {mode}", flush=True)
    opt = dict(precision=prec, norm=norm, rel_tol=1e-11, mg_cycle=cyc, mg_coarse_max=cm)
    E1, T1, i1 = _run(fld, torch, prob, 6, multi=False, **opt)
    E2, T2, i2 = _run(fld, torch, prob, 6, multi=mode, **opt)
    assert [i["status"] for i in i2] == [0] * 6
    assert [i["inner_iters"] for i in i1] == [i["inner_iters"] for i in i2]
    assert np.array_equal(E1, E2) and np.array_equal(T1, T2)


def test_steps_profiled_path_matches(lib):
    fld = lib
    prob = W.make("c2", nx=40, ny=33)
    opt = dict(precision="mixed", norm=1, rel_tol=1e-11)
    E1, T1, i1 = _run(fld, torch, prob, 4, multi=True, profile=False, **opt)
    E2, T2, i2 = _run(fld, torch, prob, 4, multi=True, profile=True, **opt)
    st = ([i["status"] for i in i1], [i["status"] for i in i2])
    assert st == ([0] * 4, [0] * 4), st
    assert np.array_equal(E1, E2) and np.array_equal(T1, T2)


@pytest.mark.parametrize("name,kw,norm,cm", [
    ("c5", dict(nx=64, ny=48), 1, 64),
    ("c3", dict(nx=40, ny=40), 0, 64),
    ("c5", dict(nx=256, ny=128), 1, 2048),
])
def test_steps_vs_oracle(lib, name, kw, norm, cm):
    """Ten coupled steps; each step's solve error (<= about 1e-12 relative) is
    carried into the next step's coefficients, so the bound is looser than a
    single step's.  (mg_coarse_max 2048: the dense coarsest level.)"""
    fld = lib
    prob = W.make(name, **kw)
    print(f"[steps vs oracle] {name} {prob.nx}x{prob.ny} coarse {cm}", flush=True)
    n = 10
    E, T, infos = _run(fld, torch, prob, n, multi=True, precision="mixed", norm=norm, rel_tol=1e-12,
                       mg_coarse_max=cm)
    assert all(i["status"] == 0 for i in infos)
    Eo, To = _oracle_steps(prob, n)
    assert rel_l2(E, Eo) < 1e-9
    assert rel_l2(T, To) < 1e-9
    assert np.max(np.abs(E - Eo) / np.abs(Eo)) < 1e-6


def test_steps_zero_and_one(lib):
    fld = lib
    prob = W.make("c1", nx=20, ny=18)
    E0, T0, inf0 = _run(fld, torch, prob, 0, multi=True)
    assert np.array_equal(E0, prob.E) and np.array_equal(T0, prob.T)
    E1, T1, _ = _run(fld, torch, prob, 1, multi=True)
    E2, T2, _ = _run(fld, torch, prob, 1, multi=False)
    assert np.array_equal(E1, E2) and np.array_equal(T1, T2)


def test_steps_budget_exhausted_is_reported(lib):
    """A budget of 2 iterations cannot converge: every step reports ENOCONV
    and the call returns it (the first step stops the run)."""
    fld = lib
    prob = W.make("c2", nx=48, ny=48)
    _, _, infos = _run(fld, torch, prob, 3, multi=True, max_inner=2)
    assert infos[0]["status"] == 4


@pytest.mark.parametrize("use_graph", [1, 0])
def test_sweep_replay_measurement(lib, use_graph):
    """fld_profile_sweeps replays one V-cycle's line sweeps (as a graph, or
    as plain launches in a context without graphs): it needs an assembled
    context, counts every grid level's band launches (four per level, levels
    above the LDS sub-cycle), selects level ranges, reports positive times
    and bytes, and leaves the next step equal to a step of a fresh context."""
    fld = lib
    prob = W.make("c2", nx=256, ny=256)
    opt = dict(precision="mixed", norm=1, rel_tol=1e-11)
    ctx = make_ctx(fld, prob, use_graph=use_graph, **opt)
    with pytest.raises(fld.FLDError):
        ctx.profile_sweeps(2)
    t = to_dev(prob, torch)
    args = (t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], prob.dt, t["ghost_E"])
    ctx.step(t["E"], t["T"], *args, check=False)
    r = ctx.profile_sweeps(5)
    # 256^2 -> sub-cycle from 64^2: levels 256 and 128 on the grid, 4 band launches each
    assert r["launches"] == 8
    assert r["us_per_launch"] > 0.0 and r["bytes_per_launch"] > 0.0
    fine, coarse = ctx.profile_sweeps(3, levels=1), ctx.profile_sweeps(3, first=1)
    assert fine["launches"] == 4 and coarse["launches"] == 4
    # the level of 128^2 cells moves a quarter of the bytes of the 256^2 level
    assert coarse["bytes_per_launch"] == pytest.approx(fine["bytes_per_launch"] / 4, rel=0.05)
    with pytest.raises(fld.FLDError):
        ctx.profile_sweeps(2, first=2)  # the sub-cycle's levels are not launched
    t2 = to_dev(prob, torch)
    info = ctx.step(t2["E"], t2["T"], *args, check=False)
    torch.cuda.synchronize()
    ctx.close()
    E_ref, T_ref, i_ref = _run(fld, torch, prob, 1, multi=False, **opt)
    assert info["status"] == 0 and info["inner_iters"] == i_ref[0]["inner_iters"]
    assert np.array_equal(t2["E"].cpu().numpy(), E_ref) and np.array_equal(t2["T"].cpu().numpy(), T_ref)


def test_steps_graph_equals_steps(lib):
    """The captured form (fld_steps_graph, called through the C ABI) and the
    pipelined form give the same fields bit for bit."""
    import ctypes
    from paper_2602_12545_amd import _binding as B
    prob = W.make("c1", nx=40, ny=32)
    E1, T1, _ = _run(lib, torch, prob, 4, multi=True, precision="mixed")
    ctx = make_ctx(lib, prob, precision="mixed")
    t = to_dev(prob, torch)
    infos = (B.fld_solve_info * 4)()
    st = B.lib.fld_steps_graph(ctx.handle, 4, B._ptr(t["E"]), B._ptr(t["T"]), B._ptr(t["rho"]), B._ptr(t["kappa_R"]),
                               B._ptr(t["kappa_P"]), B._ptr(t["c_v"]), B._ptr(t["ghost_E"]), ctypes.c_double(prob.dt),
                               infos)
    torch.cuda.synchronize()
    ctx.close()
    assert st == 0 and [infos[k].status for k in range(4)] == [0] * 4
    assert np.array_equal(t["E"].cpu().numpy(), E1) and np.array_equal(t["T"].cpu().numpy(), T1)


@pytest.mark.skip(reason="a host-side segmentation fault inside fld_steps_graph's capture and replay, after "
                         "host-driven steps on the same context, is not yet explained (the captured step's open "
                         "issue); the sequence stays off the GPU until its cause is found")
def test_host_driven_solves_refused_after_graph_replay(lib):
    """Once fld_steps_graph has replayed its captured step on a context, the
    host-driven entry points (fld_step, fld_solve, fld_steps, fld_substep)
    refuse it with EINVAL before any device work; further fld_steps_graph
    calls still run."""
    fld = lib
    prob = W.make("c1", nx=24, ny=20)
    ctx = make_ctx(fld, prob, precision="mixed")
    t = to_dev(prob, torch)
    args = (t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], prob.dt, t["ghost_E"])
    ctx.steps_graph(1, t["E"], t["T"], *args)     # the first step runs host-driven: no replay yet
    ctx.step(t["E"], t["T"], *args)
    ctx.steps_graph(3, t["E"], t["T"], *args)
    for call in (lambda: ctx.step(t["E"], t["T"], *args), lambda: ctx.steps(2, t["E"], t["T"], *args),
                 lambda: ctx.solve(t["E"]), lambda: ctx.substep(t["E"], t["T"], *args, n_sub=2)):
        with pytest.raises(fld.FLDError) as e:
            call()
        assert e.value.status == fld.FLD_EINVAL and "fld_steps_graph" in str(e.value)
    infos = ctx.steps_graph(2, t["E"], t["T"], *args)
    torch.cuda.synchronize()
    ctx.close()
    assert [i["status"] for i in infos] == [0, 0]
