"""The allocation-free block step (fld_block_step_noalloc) against the batch
step of a one-block batch: the same kernel on the same inputs, so the fields
and records agree bit for bit.  Two calls in a row share the static
workspace, the second on a smaller block (its stale contents must not leak
into the result), in every precision; both are also checked against the
oracle's step of the block."""
import numpy as np
import pytest

import fld_workloads as W
from oracle import fld_oracle as O
from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FIELDS = ("E", "T", "rho", "kappa_R", "kappa_P", "c_v", "ghost_E")


def _dev(prob):
    return {k: torch.tensor(np.ascontiguousarray(getattr(prob, k)), dtype=torch.float64, device="cuda")
            for k in FIELDS}


def _via_batch(lib, prob, opt):
    bt = lib.Batch([prob.nx], [prob.ny], [prob.x_faces[1]], [prob.y_faces[1]], None, opt)
    f = _dev(prob)
    info = bt.step(f["E"], f["T"], f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], prob.dt, f["ghost_E"],
                   check=False)[0]
    torch.cuda.synchronize()
    bt.close()
    return f["E"].cpu().numpy(), f["T"].cpu().numpy(), info


def _via_noalloc(lib, prob, opt):
    f = _dev(prob)
    info = lib.block_step_noalloc(prob.nx, prob.ny, prob.x_faces[1], prob.y_faces[1], f["E"], f["T"], f["rho"],
                                  f["kappa_R"], f["kappa_P"], f["c_v"], prob.dt, f["ghost_E"], options=opt,
                                  check=False)
    torch.cuda.synchronize()
    return f["E"].cpu().numpy(), f["T"].cpu().numpy(), info


@pytest.mark.parametrize("prec", ["mixed", "fp64", "fp32"])
def test_noalloc_equals_batch_step_twice(lib, prec):
    opt = lib.default_options(precision=prec, rel_tol=1e-12, norm=1)
    for b, (nx, ny) in ((3, (128, 96)), (4, (40, 24))):
        prob = W.make_c4_block(b, nx, ny)
        print(f"[noalloc] {prec} block {nx}x{ny}", flush=True)
        Eb, Tb, ib = _via_batch(lib, prob, opt)
        En, Tn, inn = _via_noalloc(lib, prob, opt)
        assert inn["call_status"] == ib["status"]
        if prec != "fp32":  # one binary32 solve stops at its inner tolerance, not at 1e-12
            assert ib["status"] == 0
        assert np.array_equal(En, Eb) and np.array_equal(Tn, Tb)
        for k in ("status", "outer_iters", "inner_iters", "mg_levels", "rel_resid", "rel_resid_row",
                  "rel_resid_scaled"):
            assert inn[k] == ib[k], k
        if prec != "fp32":
            r = O.step_problem(prob)
            assert rel_l2(En, r.E) < 1e-10 and rel_l2(Tn, r.T) < 1e-10


def test_noalloc_rejects_a_block_beyond_the_workspace(lib):
    opt = lib.default_options(precision="fp64")
    prob = W.make_c4_block(0, 16, 16)
    f = _dev(prob)
    with pytest.raises(lib.FLDError) as e:
        lib.block_step_noalloc(300, 300, 1e10, 1e10, f["E"], f["T"], f["rho"], f["kappa_R"], f["kappa_P"],
                               f["c_v"], prob.dt, f["ghost_E"], options=opt)
    assert e.value.status == lib.FLD_EINVAL
