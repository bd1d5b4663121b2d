"""Autotuner on the GPU: the chosen configuration converges and, used for a
step, still matches the oracle; the cache replays the choice."""
import numpy as np
import pytest

import fld_workloads as W
from oracle import fld_oracle as O
from gpu_helpers import gpu_step, rel_l2, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_tune_grid_picks_a_converging_configuration(lib, tmp_path):
    from paper_2602_12545_amd import tune
    prob = W.make_c2(nx=96, ny=80)
    f = to_dev(prob, torch)
    base = lib.default_options(precision="mixed", rel_tol=1e-12, norm=1)
    path = str(tmp_path / "t.json")
    best, table = tune.tune_grid(prob.nx, prob.ny, prob.geom, prob.x_faces, prob.y_faces,
                                 [(b.kind, b.value) for b in prob.bc], f, prob.dt, base=base, reps=1, cache=path)
    # 2 line smoothers x 5 cycles x 12 (4 coarsest sizes x 3 chunks), and
    # point smoothing x 12
    assert len(table) == 132
    assert {e["options"]["mg_coarse_max"] for e in table} == {64, 256, 1024, 4096}
    ok = [e for e in table if e["status"] == 0]
    chosen = [e for e in ok if all(e["options"][k] == getattr(best, k) for k in e["options"])]
    assert chosen and chosen[0]["ms"] == min(e["ms"] for e in ok)
    # inputs untouched by the trials
    assert np.array_equal(f["E"].cpu().numpy(), prob.E)
    opts = {k: getattr(best, k) for k in ("smoother", "mg_coarse_max", "chunk", "mg_cycle")}
    E, T, info = gpu_step(lib, torch, prob, precision="mixed", rel_tol=1e-12, norm=1, **opts)
    assert info["status"] == 0
    r = O.step_problem(prob)
    assert rel_l2(E, r.E) < 1e-10
    best2, table2 = tune.tune_grid(prob.nx, prob.ny, prob.geom, prob.x_faces, prob.y_faces,
                                   [(b.kind, b.value) for b in prob.bc], f, prob.dt, base=base, reps=1, cache=path)
    assert table2 is None
    assert {k: getattr(best2, k) for k in opts} == opts


def test_tune_batch(lib):
    from paper_2602_12545_amd import tune
    blocks = [W.make_c4_block(b, nx, ny) for b, (nx, ny) in enumerate([(32, 16), (64, 48), (16, 16), (96, 32)])]
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    f = {k: dev(np.concatenate([getattr(b, k).ravel() for b in blocks]))
         for k in ("E", "T", "rho", "kappa_R", "kappa_P", "c_v")}
    f["ghost_E"] = dev(np.concatenate([b.ghost_E for b in blocks]))
    base = lib.default_options(precision="mixed")
    best, threads, table = tune.tune_batch([b.nx for b in blocks], [b.ny for b in blocks], [1e10] * 4, [1e10] * 4,
                                           f, 1e4, base=base, reps=1, cache="")
    assert len(table) == 9 and threads in (256, 512, 1024) and best.mg_coarse_max in (16, 32, 64)
    assert all(e["status"] == 0 for e in table)
