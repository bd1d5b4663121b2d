"""Benchmark of the implicit FLD radiation step on one MI355X.

Workload (default): the 1024 x 1024 stretched Cartesian grid with lognormal
density / temperature and clipped Kramers opacity (seeded, synthetic), one
backward-Euler radiation step (assemble + multigrid-preconditioned CG to a
1e-10 relative residual + gas update) per timed step, inputs resident in HBM.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c5"])
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64", "fp32"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    return ap.parse_args()


def run_steps(fld, torch, prob, prec, steps, warmup):
    import numpy as np
    ctx = fld.Context(prob.nx, prob.ny, prob.geom, prob.x_faces, prob.y_faces,
                      [(b.kind, b.value) for b in prob.bc], fld.default_options(precision=prec))
    dev = "cuda"
    base = {k: torch.tensor(np.ascontiguousarray(getattr(prob, k)), dtype=torch.float64, device=dev)
            for k in ("E", "T", "rho", "kappa_R", "kappa_P", "c_v")}
    E = base["E"].clone()
    T = base["T"].clone()
    infos = []

    def one():
        E.copy_(base["E"])
        T.copy_(base["T"])
        return ctx.step(E, T, base["rho"], base["kappa_R"], base["kappa_P"], base["c_v"], prob.dt)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infos.append(one())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    return dt / steps, infos


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is described in DESIGN.md"}))
        sys.exit(2)
    import torch
    import paper_2602_12545_amd as fld
    import fld_workloads as W

    prob = W.make(args.workload)
    ncell = prob.nx * prob.ny
    ms_mixed, infos = run_steps(fld, torch, prob, args.precision, args.steps, args.warmup)
    iters = sum(i["inner_iters"] for i in infos) / len(infos)
    out = {
        "metric": "FLD solves/s & Mcell-iter/s to 1e-10 resid; HBM GB/s %peak; mixed vs FP64",
        "value": 1.0 / ms_mixed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_mixed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "f32+f64", "fp64": "f64", "fp32": "f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {prob.nx}x{prob.ny} "
                               + ("stretched Cartesian" if prob.geom == 0 else "spherical-polar"),
                   "cells": ncell, "precision": args.precision, "rel_tol": 1e-10},
        "inner_iters": iters,
        "mcell_iter_per_s": ncell * iters / ms_mixed / 1e6,
        "final_rel_resid": max(i["rel_resid"] for i in infos),
        "status": sorted(set(i["status"] for i in infos)),
    }
    if not args.no_fp64 and args.precision != "fp64":
        ms64, infos64 = run_steps(fld, torch, prob, "fp64", max(3, args.steps // 2), 1)
        out["fp64_ms_per_step"] = ms64 * 1e3
        out["fp64_inner_iters"] = sum(i["inner_iters"] for i in infos64) / len(infos64)
        out["mixed_vs_fp64_speedup"] = ms64 / ms_mixed
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
