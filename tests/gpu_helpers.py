"""Helpers for the GPU tests: run a workload through the C ABI binding."""
import numpy as np

FIELDS = ("E", "T", "rho", "kappa_R", "kappa_P", "c_v")


def to_dev(prob, torch):
    t = {k: torch.tensor(np.ascontiguousarray(getattr(prob, k)), dtype=torch.float64, device="cuda") for k in FIELDS}
    t["ghost_E"] = (torch.tensor(prob.ghost_E, dtype=torch.float64, device="cuda")
                    if prob.ghost_E is not None else None)
    return t


def make_ctx(fld, prob, **opt):
    return fld.Context(prob.nx, prob.ny, prob.geom, prob.x_faces, prob.y_faces,
                       [(b.kind, b.value) for b in prob.bc], fld.default_options(**opt))


def gpu_step(fld, torch, prob, **opt):
    ctx = make_ctx(fld, prob, **opt)
    t = to_dev(prob, torch)
    info = ctx.step(t["E"], t["T"], t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], prob.dt, t["ghost_E"],
                    check=False)
    torch.cuda.synchronize()
    out = t["E"].cpu().numpy(), t["T"].cpu().numpy(), info
    ctx.close()
    return out


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
