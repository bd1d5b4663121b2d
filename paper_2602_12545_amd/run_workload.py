"""Run one seeded workload's implicit step repeatedly on cuda:0 and print the
time per step as one JSON line: a driver for profilers (rocprofv3 traces one
workload at a time, with no tuning search in the trace).

    python -m paper_2602_12545_amd.run_workload c2 --precision mixed --reps 10 \
        --smoother line --mg-cycle k --mg-coarse-max 256 --chunk 4
    python -m paper_2602_12545_amd.run_workload c4 --precision mixed --threads 512

c1, c2 and c3 are single grids stepped through one context (Section 3.2.1,
one implicit step: assembly, solve, gas update); c4 is the batch of
independent ghost-bounded blocks (Section 3.2.2) stepped by one launch.  Each
repetition restarts from the workload's initial state.
"""
from __future__ import annotations

import argparse
import json
import time

SMOOTHERS = {"line": 0, "point": 1, "line_split": 2}
CYCLES = {"v": 0, "k": 1, "w2": 2, "kl_k": 3, "kl_w2": 4}
FIELDS = ("E", "T", "rho", "kappa_R", "kappa_P", "c_v")


def _parse(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("workload", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64", "fp32"])
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--norm", type=int, default=None, help="0 per-volume rows, 1 Jacobi-scaled (default: "
                                                            "the workload's: scaled for the spherical c3)")
    ap.add_argument("--rel-tol", type=float, default=1e-10)
    ap.add_argument("--smoother", choices=list(SMOOTHERS), default=None)
    ap.add_argument("--mg-cycle", choices=list(CYCLES), default=None)
    ap.add_argument("--mg-coarse-max", type=int, default=None)
    ap.add_argument("--chunk", type=int, default=None)
    ap.add_argument("--threads", type=int, default=512, help="batch workgroup size (c4)")
    return ap.parse_args(argv)


def main(argv=None):
    a = _parse(argv)
    import numpy as np
    import torch
    import fld_workloads as W
    from . import Batch, Context, default_options

    prob = W.make(a.workload)
    norm = a.norm if a.norm is not None else (1 if a.workload == "c3" else 0)
    kw = dict(precision=a.precision, norm=norm, rel_tol=a.rel_tol)
    if a.smoother is not None:
        kw["smoother"] = SMOOTHERS[a.smoother]
    if a.mg_cycle is not None:
        kw["mg_cycle"] = CYCLES[a.mg_cycle]
    if a.mg_coarse_max is not None:
        kw["mg_coarse_max"] = a.mg_coarse_max
    if a.chunk is not None:
        kw["chunk"] = a.chunk
    opt = default_options(**kw)
    dev = lambda v: torch.tensor(np.ascontiguousarray(v), dtype=torch.float64, device="cuda")
    if a.workload == "c4":
        blocks = prob.blocks
        f = {k: dev(prob.packed(k)) for k in FIELDS}
        ghost = dev(prob.packed_ghosts())
        dx = [b.x_faces[1] - b.x_faces[0] for b in blocks]
        dy = [b.y_faces[1] - b.y_faces[0] for b in blocks]
        solver = Batch([b.nx for b in blocks], [b.ny for b in blocks], dx, dy, None, opt)
        solver.threads = a.threads
        dt, cells = blocks[0].dt, sum(b.nx * b.ny for b in blocks)

        def step(E, T):
            return solver.step(E, T, f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], dt, ghost, check=False)
    else:
        f = {k: dev(getattr(prob, k)) for k in FIELDS}
        ghost = dev(prob.ghost_E) if prob.ghost_E is not None else None
        solver = Context(prob.nx, prob.ny, prob.geom, prob.x_faces, prob.y_faces,
                         [(b.kind, b.value) for b in prob.bc], opt)
        dt, cells = prob.dt, prob.nx * prob.ny

        def step(E, T):
            return [solver.step(E, T, f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], dt, ghost)]
    E, T = f["E"].clone(), f["T"].clone()
    step(E, T)  # warm-up: first launches, graph capture
    torch.cuda.synchronize()
    ts = []
    for _ in range(a.reps):
        E.copy_(f["E"])
        T.copy_(f["T"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = step(E, T)
        torch.cuda.synchronize()
        ts.append(1e3 * (time.perf_counter() - t0))
    solver.close()
    its = [i["inner_iters"] for i in infos]
    print(json.dumps({"workload": a.workload, "cells": cells, "precision": a.precision, "reps": a.reps,
                      "ms_per_step_median": float(np.median(ts)), "ms_per_step_min": min(ts),
                      "inner_iters_max": max(its), "inner_iters_mean": sum(its) / len(its),
                      "status": sorted(set(i["status"] for i in infos)), "options": kw}), flush=True)


if __name__ == "__main__":
    main()
