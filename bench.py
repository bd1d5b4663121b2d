"""Benchmark of the implicit FLD radiation step on one MI355X.

Headline workload: the 4096 x 2048 spherical-polar stress recipe (r log-spaced
1e11 .. 1e14 cm, theta 0 .. pi; lognormal opacity with sigma_ln 4, contrast
1e8; c_v = 1e6, dt = 1e5 s), run as consecutive implicit steps through
fld_steps (steps queued back to back, CG iterations in captured two-slot
chunks whose solver flags the host reads one chunk behind; T updated from the
linearised exchange every step, opacities fixed).  One benchmark step = one
implicit radiation step of that sequence (assembly, multigrid-preconditioned
CG with FP32 inner iterations and FP64 reliable updates to a 1e-10 relative
residual in the Jacobi-scaled norm, gas update), inputs resident in HBM.
The W warm-up steps run as one fld_steps call from the initial state; the K
timed steps as one fld_steps call from the initial state again.  The whole
100-step sequence is then run as one fld_steps call per precision (mixed and
FP64, each on the fastest of its multigrid cycles, KL_W2, KL_K, W2 and K,
chosen by a three-step probe), which gives time-to-1e-10 per step and the
mixed/FP64 ratio; the K timed steps are also run in FP64.  Prints one JSON
line.

Beyond the contract's fields: the dominant kernel's roofline (the coarse
levels' band-fused line sweeps, replayed between HIP events, with the finest
level's half-sweeps beside it), the other
workloads (64 x 64 FP64 solves/s; 1024 x 1024 stretched Cartesian and
2048 x 512 spherical steps, mixed, FP64 and FP32-only; 256 batched blocks),
the relative L2 error of E and T against the CPU oracle per workload (full
size for the 64 x 64, 1024 x 1024 and 2048 x 512 grids and the 256 blocks, a
full-resolution 4096 x 256 theta slab for the stress grid), the sub-cycled
step and advection, and cpu_baseline: the oracle timed on the host's cores
on the headline grid cut into one decoupled theta slab per core.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure
METRIC = "FLD solves/s & Mcell-iter/s to 1e-10 resid; HBM GB/s %peak; mixed vs FP64"
FIELDS = ("E", "T", "rho", "kappa_R", "kappa_P", "c_v")
SEQUENCE = 100          # steps of the stress workload
CYCLES = {"v": 0, "k": 1, "w2": 2, "kl_k": 3, "kl_w2": 4}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--mg-cycle", default=None, choices=list(CYCLES),
                    help="fix the multigrid cycle of the stress workload (default: the fastest of KL_W2, KL_K, "
                         "W2 and K by a three-step probe, per precision)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 runs of the stress steps")
    ap.add_argument("--no-sequence", action="store_true", help="skip the 100-step runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the other workloads")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the comparisons with the oracle")
    ap.add_argument("--no-profile", action="store_true", help="no replay measurement (no roofline)")
    ap.add_argument("--no-graph", action="store_true",
                    help="run the stress steps as plain launches (use_graph = 0; for HBM counter passes, which do "
                         "not survive the multi-step graphs under rocprofv3 --pmc)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device copy 5 times (scale for HBM traffic counters)")
    return ap.parse_args()


def dev_fields(torch, prob):
    import numpy as np
    f = {k: torch.tensor(np.ascontiguousarray(getattr(prob, k)), dtype=torch.float64, device="cuda") for k in FIELDS}
    f["ghost_E"] = (torch.tensor(prob.ghost_E, dtype=torch.float64, device="cuda")
                    if prob.ghost_E is not None else None)
    return f


def rel_l2(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def kernel_source_digest():
    """Digest of the measured kernels and their launches: the multigrid and
    band headers that define k_line and k_band, the headers they include, and
    the host functions that pick their chunking and launch them (comments and
    white space removed).  HBM traffic counters taken on other code no longer
    describe the line sweeps; host changes elsewhere leave them valid."""
    import hashlib
    import re
    d = os.path.join(ROOT, "paper_2602_12545_amd", "csrc")
    h = hashlib.sha1()

    def clean(src):
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        return re.sub(r"\s+", "", src)

    for f in ("fld_internal.hpp", "fld_kernels.hpp", "fld_line.hpp", "fld_mg.hpp", "fld_sub.hpp", "fld_band.hpp"):
        h.update(f.encode())
        h.update(clean(open(os.path.join(d, f)).read()).encode())
    host = open(os.path.join(d, "fld_host.hip")).read()
    for fn in ("inline void line_params", "int launch_line", "int launch_band"):
        i = host.index(fn)
        j = host.index("\n}\n", i)
        h.update(clean(host[i:j]).encode())
    return h.hexdigest()[:16]


def measured_traffic(name):
    """HBM bytes per launch from a committed counter summary, if it was taken
    on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None, "no counter summary"
    vals = {}
    for line in open(path):
        line = line.strip().strip("`")
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_digest") != kernel_source_digest():
        return None, "counters taken on other kernel sources"
    try:
        return float(vals["traffic_bytes_per_launch"]), "profiles/" + name
    except (KeyError, ValueError):
        return None, "counter summary incomplete"


def make_ctx(fld, prob, opt):
    return fld.Context(prob.nx, prob.ny, prob.geom, prob.x_faces, prob.y_faces,
                       [(b.kind, b.value) for b in prob.bc], opt)


NO_GRAPH = False


def stress_options(fld, prec, cycle):
    # coarsest level 64 x 32 (2048 cells): solved exactly with its dense
    # inverse (multi-workgroup product) instead of the one-workgroup sub-cycle
    return fld.default_options(precision=prec, norm=1, rel_tol=1e-10, mg_cycle=cycle, mg_coarse_max=2048,
                               use_graph=0 if NO_GRAPH else 1)


def run_sequence(fld, torch, prob, f, opt, nsteps, ctx=None):
    """nsteps consecutive steps from the initial state as one fld_steps call:
    wall time per step (host clock around the call, stream synchronised) and
    the per-step records."""
    own = ctx is None
    ctx = ctx or make_ctx(fld, prob, opt)
    E, T = f["E"].clone(), f["T"].clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = ctx.steps(nsteps, E, T, f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], prob.dt, f["ghost_E"],
                      check=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if own:
        ctx.close()
    return dt / nsteps, infos, (E, T)


def summarise(prob, ms, infos):
    import numpy as np
    its = [i["inner_iters"] for i in infos]
    return {"ms_per_step": ms, "solves_per_s": 1e3 / ms, "iters_mean": float(np.mean(its)), "iters_max": max(its),
            "iters_min": min(its), "status": sorted(set(i["status"] for i in infos)),
            "max_rel_resid": max(i["rel_resid"] for i in infos),
            "mcell_iter_per_s": prob.nx * prob.ny * float(np.mean(its)) / (ms * 1e-3) / 1e6}


def pick_cycle(fld, torch, prob, f, prec, fixed):
    """The fastest of the K-cycle, two sequential V-cycles and their
    Krylov-accelerated variants on three steps of the stress sequence (after
    one warm-up step), unless fixed."""
    if fixed is not None:
        return CYCLES[fixed], None
    probe = {}
    for name in ("kl_w2", "kl_k", "w2", "k"):
        ctx = make_ctx(fld, prob, stress_options(fld, prec, CYCLES[name]))
        run_sequence(fld, torch, prob, f, None, 1, ctx)
        ms, infos, _ = run_sequence(fld, torch, prob, f, None, 3, ctx)
        ctx.close()
        ok = all(i["status"] == 0 for i in infos)
        probe[name] = {"ms_per_step": 1e3 * ms, "ok": ok}
    good = [n for n in probe if probe[n]["ok"]] or list(probe)
    best = min(good, key=lambda n: probe[n]["ms_per_step"])
    return CYCLES[best], probe


def roofline(ctx, reps=50):
    """The dominant kernel of the stress step: the band-fused zebra line
    sweeps (`k_band`, both colours of one direction per launch) of grid
    levels 1 .. 5, the largest share of the step's kernel time (the finest
    level's `k_line` half-sweeps, the LDS sub-cycle and the Krylov-level
    kernels follow).  One V-cycle's line-sweep launches of those levels are
    captured on a solver state that never converges and replayed between two
    HIP events on the solve stream; the time per launch includes the gap
    between dependent launches (the same time minus that of an equal graph of
    empty launches, which also removes the empty kernels' own execution, is
    reported as an upper bound).  The finest level's half-sweeps, the
    bandwidth-bound kernel, are measured alike and reported beside it."""
    def measure(rep, pmc):
        us = rep["us_per_launch"]
        traffic, tnote = measured_traffic(pmc)
        return {"achieved": rep["bytes_per_launch"] / (us * 1e-6) / 1e9, "avg_launch_us": us,
                "bytes_per_launch": rep["bytes_per_launch"], "traffic": traffic, "traffic_source": tnote,
                "replay": rep, "upper_bound_minus_empty_launches": rep["bytes_per_launch"] / (
                    max(us - rep["floor_us"], 1e-3) * 1e-6) / 1e9}
    fine = measure(ctx.profile_sweeps(reps, levels=1), "pmc_c5_fine_line_sweeps.md")
    band = measure(ctx.profile_sweeps(reps, first=1), "pmc_c5_band_sweeps.md")
    out = {"bound": "hbm", "achieved": band["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": band["achieved"] / HBM_PEAK_GBS, "traffic": band["traffic"],
           "kernel": "k_band on grid levels 1-5 (2048x1024 .. 128x64): band-fused zebra line sweeps, both colours "
                     "of one direction per launch; the largest share of the stress step's kernel time",
           "duration_method": f"graph replay of one V-cycle's {band['replay']['launches']} line-sweep launches on "
                              f"levels 1-5 x {reps}, HIP events on the solve stream, per-launch time with the "
                              "launch gaps",
           **{k: band[k] for k in ("avg_launch_us", "bytes_per_launch", "traffic_source", "replay",
                                   "upper_bound_minus_empty_launches")}}
    out["fine_level_line_sweeps"] = {
        "kernel": "k_line on the finest level (4096x2048): the zebra line half-sweeps of both directions",
        "frac": fine["achieved"] / HBM_PEAK_GBS, **fine}
    return out


def _oracle_slab_step(prob):
    """One oracle step of one slab on one core (a worker process): wall-clock
    start and end of the step, after a warm-up."""
    from threadpoolctl import threadpool_limits
    from oracle import fld_oracle as O
    import fld_workloads as W
    with threadpool_limits(limits=1):
        O.step_problem(W.make_c2(nx=64, ny=64))  # warm-up (imports, allocator)
        t0 = time.time()
        O.step_problem(prob)
        t1 = time.time()
    return t0, t1


def cpu_baseline(W, max_procs=16):
    """The CPU oracle as it stands (FP64 assembly, SuperLU direct solve with
    extended-precision refinement, gas update; single-threaded) on the host's
    cores: the stress grid cut into as many theta slabs at full resolution as
    there are cores (up to max_procs), one oracle step per slab, the slabs in
    parallel worker processes (one core each).  The cut slabs are decoupled
    (reflecting cut sides), which flatters the CPU: the direct solve of the
    whole grid costs more than that of its slabs."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    cores = len(os.sched_getaffinity(0))
    nproc = max(1, min(max_procs, cores))
    c5 = W.make_c5()
    cuts = [round(k * c5.ny / nproc) for k in range(nproc + 1)]
    slabs = [W.theta_slab(c5, cuts[k], cuts[k + 1]) for k in range(nproc)]
    shape = f"{c5.nx}x{c5.ny}"
    del c5
    with ProcessPoolExecutor(max_workers=nproc, mp_context=multiprocessing.get_context("spawn")) as ex:
        spans = list(ex.map(_oracle_slab_step, slabs))
    wall = max(t1 for _, t1 in spans) - min(t0 for t0, _ in spans)
    slow = max(t1 - t0 for t0, t1 in spans)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": 1.0 / wall, "unit": "solves/s", "cores": nproc, "kind": "oracle",
            "sample": f"one oracle step of the stress recipe's {shape} grid cut into {nproc} decoupled theta slabs "
                      f"of {shape.split('x')[0]}x{c5_rows(cuts)} cells, solved concurrently by {nproc} single-threaded processes: "
                      f"{wall:.1f} s from the first slab's start to the last one's end (slowest slab {slow:.1f} s); "
                      f"one step of the whole grid's cells per {wall:.1f} s (flatters the CPU: the slabs are decoupled "
                      f"and the direct solve grows faster than linearly)",
            "host_cores": cores, "cpu_model": model}


def c5_rows(cuts):
    """Slab heights as text ('256' when equal, else 'min-max')."""
    h = [b - a for a, b in zip(cuts[:-1], cuts[1:])]
    return str(h[0]) if min(h) == max(h) else f"{min(h)}-{max(h)}"


def single_step_line(fld, torch, prob, opt, reps):
    """Median wall time of one step restored from the same initial state (each
    step timed on its own, between synchronisations; the restoring copies are
    outside the timed interval)."""
    import statistics
    f = dev_fields(torch, prob)
    ctx = make_ctx(fld, prob, opt)
    E, T = f["E"].clone(), f["T"].clone()

    def one():
        E.copy_(f["E"])
        T.copy_(f["T"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ctx.step(E, T, f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], prob.dt, f["ghost_E"], check=False)
        torch.cuda.synchronize()
        return info, 1e3 * (time.perf_counter() - t0)

    one()
    runs = [one() for _ in range(reps)]
    infos = [r[0] for r in runs]
    ms = statistics.median(r[1] for r in runs)
    ctx.close()
    return ms, infos, (E.cpu().numpy(), T.cpu().numpy())


def other_workloads(fld, torch, W, tuner, accuracy):
    """64 x 64 FP64 solves/s; the 1024 x 1024 and 2048 x 512 grids in mixed,
    FP64 and FP32-only precision (every schedule autotuned per precision);
    each against the oracle when accuracy is set."""
    from oracle import fld_oracle as O
    out = {}
    # (label, precision, norm, rel_tol, reps): the metric's 1e-10 stop and, on
    # the 1024 x 1024 grid, a tighter stop at which the error meets 1e-10 too
    # (a 1e-10 residual bounds the error only up to the conditioning)
    jobs = [("c1", W.make_c1(), [("fp64", "fp64", 0, 1e-10, 200)], "tune"),
            ("c2", W.make_c2(), [("mixed", "mixed", 0, 1e-10, 10), ("fp64", "fp64", 0, 1e-10, 5),
                                 ("mixed_stop_2e-11", "mixed", 0, 2e-11, 10), ("fp64_stop_2e-11", "fp64", 0, 2e-11, 5),
                                 ("fp32", "fp32", 0, 1e-10, 5)], "tune"),
            ("c3", W.make_c3(), [("mixed", "mixed", 1, 1e-10, 10), ("fp64", "fp64", 1, 1e-10, 5),
                                 ("fp32", "fp32", 1, 1e-10, 5)], "tune")]
    for name, prob, runs, tune in jobs:
        f = dev_fields(torch, prob)
        ref = O.step_problem(prob) if accuracy else None
        geom = "stretched Cartesian" if prob.geom == 0 else "spherical-polar"
        res = {"workload": f"{name}: {prob.nx}x{prob.ny} {geom}, one implicit step"}
        # each precision on its own tuned schedule (binary64 cannot hold the
        # same coarse levels in LDS, so its best schedule differs); the
        # binary32-only runs take the mixed-precision one
        tuned = {}
        if tune and tuner is not None:
            for tp in sorted({"fp64" if r[1] == "fp64" else "mixed" for r in runs}):
                tuned[tp], _ = tuner.tune_grid(prob.nx, prob.ny, prob.geom, prob.x_faces, prob.y_faces,
                                               [(b.kind, b.value) for b in prob.bc], f, prob.dt,
                                               base=fld.default_options(precision=tp, norm=runs[0][2]),
                                               reps=1, cache="")
        for label, prec, norm, tol, reps in runs:
            opt = fld.default_options(precision=prec, norm=norm, rel_tol=tol)
            sched = tuned.get("fp64" if prec == "fp64" else "mixed")
            if sched is not None:
                for k in ("smoother", "mg_coarse_max", "mg_coarse_op", "chunk", "mg_cycle"):
                    setattr(opt, k, getattr(sched, k))
            ms, infos, (E, T) = single_step_line(fld, torch, prob, opt, reps)
            r = {"ms_per_step": ms, "solves_per_s": 1e3 / ms, "inner_iters": infos[-1]["inner_iters"],
                 "rel_resid": infos[-1]["rel_resid"], "status": infos[-1]["status"], "rel_tol": tol,
                 "norm": "per-volume rows" if norm == 0 else "Jacobi-scaled",
                 "mcell_iter_per_s": prob.nx * prob.ny * infos[-1]["inner_iters"] / (ms * 1e-3) / 1e6}
            if ref is not None:
                r["rel_l2_E"] = rel_l2(E, ref.E)
                r["rel_l2_T"] = rel_l2(T, ref.T)
            res[label] = r
        if "mixed" in res and "fp64" in res:
            res["mixed_vs_fp64"] = res["fp64"]["ms_per_step"] / res["mixed"]["ms_per_step"]
        for tp, sched in tuned.items():
            res["schedule" if tp == "mixed" else f"schedule_{tp}"] = {
                k: getattr(sched, k) for k in ("smoother", "mg_coarse_max", "chunk", "mg_cycle")}
        out[name] = res
    return out


def stress_slab_accuracy(fld, torch, W, cycles):
    """The headline schedule (scaled norm 1e-10, each precision's cycle) on a
    full-resolution 4096 x 256 equatorial theta slab of the stress grid, one
    step, against the oracle."""
    from oracle import fld_oracle as O
    prob = W.theta_slab(W.make_c5(), 896, 1152)
    ref = O.step_problem(prob)
    out = {"workload": "c5 theta slab rows 896..1151 (4096x256), one step"}
    for prec, cyc in cycles.items():
        ms, infos, (E, T) = single_step_line(fld, torch, prob, stress_options(fld, prec, cyc), 1)
        out[prec] = {"rel_l2_E": rel_l2(E, ref.E), "rel_l2_T": rel_l2(T, ref.T), "status": infos[-1]["status"],
                     "inner_iters": infos[-1]["inner_iters"], "rel_resid": infos[-1]["rel_resid"]}
    return out


def batch_accuracy(fld, torch, W, norm=0, rel_tol=1e-10):
    """All 256 blocks of the batched recipe (mixed, library defaults, the given
    stop), each against its own oracle step."""
    import numpy as np
    from oracle import fld_oracle as O
    batch = W.make_c4()
    blocks = batch.blocks
    dev = {k: torch.tensor(batch.packed(k), dtype=torch.float64, device="cuda")
           for k in ("E", "T", "rho", "kappa_R", "kappa_P", "c_v", "ghost_E")}
    bt = fld.Batch([b.nx for b in blocks], [b.ny for b in blocks], [1e10] * len(blocks), [1e10] * len(blocks), None,
                   fld.default_options(precision="mixed", norm=norm, rel_tol=rel_tol))
    infos = bt.step(dev["E"], dev["T"], dev["rho"], dev["kappa_R"], dev["kappa_P"], dev["c_v"], 1e4, dev["ghost_E"],
                    check=False)
    torch.cuda.synchronize()
    bt.close()
    E, T = dev["E"].cpu().numpy(), dev["T"].cpu().numpy()
    eE, eT, o = [], [], 0
    for b in blocks:
        n = b.nx * b.ny
        r = O.step_problem(b)
        eE.append(rel_l2(E[o:o + n].reshape(b.ny, b.nx), r.E))
        eT.append(rel_l2(T[o:o + n].reshape(b.ny, b.nx), r.T))
        o += n
    return {"blocks": len(blocks), "stop": f"{'Jacobi-scaled' if norm else 'per-volume rows'} {rel_tol:g}",
            "max_rel_l2_E": max(eE), "max_rel_l2_T": max(eT),
            "median_rel_l2_E": float(np.median(eE)), "status": sorted(set(i["status"] for i in infos))}


def batch_extra(fld, torch, W, tune):
    """256 independent blocks (16..128 cells per side), one launch per step."""
    import numpy as np
    batch = W.make_c4()
    blocks = batch.blocks
    nx, ny = [b.nx for b in blocks], [b.ny for b in blocks]
    d = [1e10] * len(blocks)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    f = {k: dev(batch.packed(k)) for k in FIELDS}
    f["ghost_E"] = dev(batch.packed_ghosts())
    out = {"workload": "c4: 256 Cartesian blocks, sides in {16..128}, 984320 cells, ghost boundaries"}

    def timed(prec, reps=10, norm=0, rel_tol=1e-10):
        base = defaults(fld, precision=prec, norm=norm, rel_tol=rel_tol)
        threads = 512
        if tune is not None:
            o, threads, _ = tune.tune_batch(nx, ny, d, d, f, 1e4, base=base, reps=1, cache="")
            base = o
        bt = fld.Batch(nx, ny, d, d, None, base)
        bt.threads = threads
        E, T = f["E"].clone(), f["T"].clone()

        def one(rec=False):
            E.copy_(f["E"])
            T.copy_(f["T"])
            return bt.step(E, T, f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], 1e4, f["ghost_E"], records=rec)

        one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            one()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        infos = one(True)
        bt.close()
        return ms, infos, threads, base.mg_coarse_max

    ms_m, inf_m, th_m, cm_m = timed("mixed")
    ms_d, inf_d, th_d, cm_d = timed("fp64")
    # the stop at which every block's error meets 1e-10 (Jacobi-scaled 1e-12)
    ms_mt, inf_mt, _, _ = timed("mixed", norm=1, rel_tol=1e-12)
    ms_dt, inf_dt, _, _ = timed("fp64", norm=1, rel_tol=1e-12)
    out["stop_scaled_1e-12"] = {"mixed_ms_per_step": ms_mt, "fp64_batched_ms_per_step": ms_dt,
                                "mixed_vs_fp64_batched": ms_dt / ms_mt,
                                "mixed_mean_iters": float(np.mean([i["inner_iters"] for i in inf_mt])),
                                "status": sorted(set(i["status"] for i in inf_mt + inf_dt))}
    out.update({"mixed_ms_per_step": ms_m, "mixed_tuned": {"threads": th_m, "mg_coarse_max": cm_m},
                "fp64_batched_ms_per_step": ms_d, "fp64_tuned": {"threads": th_d, "mg_coarse_max": cm_d},
                "mixed_vs_fp64_batched": ms_d / ms_m,
                "mixed_solves_per_s": len(blocks) / (ms_m * 1e-3),
                "mixed_mean_iters": float(np.mean([i["inner_iters"] for i in inf_m])),
                "status": sorted(set(i["status"] for i in inf_m + inf_d))})
    # FP64 baseline without batching: one single-grid context per block,
    # blocks stepped one after another
    ctxs, fs = [], []
    for b in blocks:
        ctxs.append(fld.Context(b.nx, b.ny, b.geom, b.x_faces, b.y_faces, [(c.kind, c.value) for c in b.bc],
                                defaults(fld, precision="fp64")))
        fs.append(dev_fields(torch, b))
    for c, g, b in zip(ctxs, fs, blocks):
        c.step(g["E"].clone(), g["T"].clone(), g["rho"], g["kappa_R"], g["kappa_P"], g["c_v"], b.dt, g["ghost_E"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, g, b in zip(ctxs, fs, blocks):
        c.step(g["E"].clone(), g["T"].clone(), g["rho"], g["kappa_R"], g["kappa_P"], g["c_v"], b.dt, g["ghost_E"])
    torch.cuda.synchronize()
    ms_pb = 1e3 * (time.perf_counter() - t0)
    for c in ctxs:
        c.close()
    out["fp64_per_block_launch_ms_per_step"] = ms_pb
    out["mixed_batched_vs_fp64_per_block"] = ms_pb / ms_m
    return out


def substep_extra(fld, torch, W, tuned):
    """Sub-cycled radiation step (fld_substep) on the 1024 x 1024 stretched
    Cartesian recipe with the gas temperature perturbed by a uniform +-30 %
    (seeded; the recipe itself starts in equilibrium, where the coupling does
    not limit): one full step as a geometric series of 4 sub-steps (q = 1.5),
    and the first 100 coupling-limited sub-steps with dbar = 0.1 (the whole
    step needs ~2350 there); the same geometric series with the power-law heat
    capacity c_v (T / T_mean)^-0.5 recomputed before every sub-step
    (fld_set_cv_law; with a positive exponent the coldest cells' small heat
    capacity lets the linearised gas update overshoot without bound on this
    stiff recipe, in the oracle too).  Wall times on the solve stream's host clock."""
    import numpy as np
    prob = W.make_c2()
    prob.T = prob.T * (1.0 + 0.3 * np.random.default_rng(11).uniform(-1.0, 1.0, prob.T.shape))
    f = dev_fields(torch, prob)
    out = {"workload": "c2 recipe (1024x1024) with T perturbed +-30 %, step dt = 1e4 in sub-steps"}
    ctx = fld.Context(prob.nx, prob.ny, prob.geom, prob.x_faces, prob.y_faces, [(b.kind, b.value) for b in prob.bc],
                      options(fld, "mixed", tuned))
    for name, kw in (("geometric_n4_q1.5", dict(n_sub=4, q=1.5, max_sub=4)),
                     ("coupling_dbar0.1_first100", dict(dbar=0.1, max_sub=100)),
                     ("geometric_n4_q1.5_cv_law_p-0.5", dict(n_sub=4, q=1.5, max_sub=4))):
        law = name.endswith("cv_law_p-0.5")
        ctx.set_cv_law(float(prob.T.mean()) if law else 1.0, -0.5 if law else 0.0)
        ms, res = [], None
        for rep in range(2):
            E, T = f["E"].clone(), f["T"].clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ctx.substep(E, T, f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], prob.dt, check=False, **kw)
            torch.cuda.synchronize()
            ms.append(1e3 * (time.perf_counter() - t0))
        n = len(res["dts"])
        out[name] = {"ms": ms[-1], "sub_steps": n, "ms_per_sub_step": ms[-1] / n,
                     "inner_iters": sum(i["inner_iters"] for i in res["infos"]),
                     "dt_covered": sum(res["dts"]) / prob.dt, "status": res["status"]}
    ctx.set_cv_law(1.0, 0.0)
    ctx.close()
    return out


def advection_extra(fld, torch, W, tuned):
    """Radiation advection (fld_set_mass_flux): the dynamical-diffusion test
    (1024 cells on [-2, 14] cm, v = 1.8 km/s, rho kappa_R = 1e7 / cm,
    kappa_P = 0, CFL 1, 714 steps to t = 6.2e-5 s) as one fld_steps call, its
    L1 error against the analytic moving Gaussian; and the 1024 x 1024
    stretched Cartesian step with a uniform +x mass flux (|f| dt dS / dV at
    most 0.5 rho)."""
    import numpy as np
    out = {}
    N, v, sig, E0 = 1024, 1.8e5, 1e7, 2e5
    xf = np.linspace(-2.0, 14.0, N + 1)
    dx = xf[1] - xf[0]
    xc = 0.5 * (xf[1:] + xf[:-1])
    one = np.ones((1, N))
    prob = W.Problem("e4", W.GEOM_CARTESIAN, xf, np.array([0.0, 1.0]),
                     np.where(np.abs(xc) < dx, E0 / (2 * dx), 1.0)[None, :], 0.1 * one, one.copy(), sig * one,
                     0.0 * one, one.copy(), dx / v, [W.BC()] * 4)
    n = int(round(6.2e-5 / prob.dt))
    f = dev_fields(torch, prob)
    fx = torch.full((1, N + 1), v, dtype=torch.float64, device="cuda")
    fy = torch.zeros((2, N), dtype=torch.float64, device="cuda")
    ctx = fld.Context(prob.nx, prob.ny, prob.geom, prob.x_faces, prob.y_faces, [(b.kind, b.value) for b in prob.bc],
                      defaults(fld, precision="mixed", norm=1, rel_tol=1e-12))
    ctx.set_mass_flux(fx, fy)
    E, T = f["E"].clone(), f["T"].clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = ctx.steps(n, E, T, f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], prob.dt, check=False)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0)
    ctx.close()
    tt = n * prob.dt
    D = 2.99792458e10 / (3 * sig)
    Ea = 1 + E0 / np.sqrt(4 * D * np.pi * tt) * np.exp(-(xc - v * tt) ** 2 / (4 * D * tt))
    Eg = E.cpu().numpy()[0]
    out["dynamical_diffusion_1024"] = {"steps": n, "ms_total": ms, "ms_per_step": ms / n,
                                       "l1_error_vs_analytic": float(np.sum(np.abs(Eg - Ea)) / np.sum(Ea - 1)),
                                       "status": sorted(set(i["status"] for i in infos))}
    prob = W.make_c2()
    f = dev_fields(torch, prob)
    ny, nx = prob.E.shape
    dxs = np.diff(prob.x_faces)
    fxv = np.broadcast_to((0.5 * float(np.median(prob.rho)) * float(dxs.min()) / prob.dt), (ny, nx + 1))
    ctx = fld.Context(prob.nx, prob.ny, prob.geom, prob.x_faces, prob.y_faces, [(b.kind, b.value) for b in prob.bc],
                      options(fld, "mixed", tuned))
    ctx.set_mass_flux(torch.tensor(np.ascontiguousarray(fxv), dtype=torch.float64, device="cuda"), None)
    ms = []
    for rep in range(4):
        E, T = f["E"].clone(), f["T"].clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ctx.step(E, T, f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], prob.dt, check=False)
        torch.cuda.synchronize()
        ms.append(1e3 * (time.perf_counter() - t0))
    ctx.close()
    out["c2_with_flux"] = {"ms_per_step": float(np.min(ms[1:])), "inner_iters": info["inner_iters"],
                           "status": info["status"]}
    return out


def copy_calibration(torch):
    n = 512 * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": 4 * n, "launches": 5}), flush=True)


def forest_extra(fld, torch, accuracy, nx0=256, ny0=256):
    """A statically refined forest solved as one matrix (fld_forest_step):
    a 256 x 256 level-0 domain (1e10 cm cells), a level-1 patch over its
    middle half and a level-2 patch over the middle half of that; fields as
    the 1024 x 1024 recipe's (lognormal rho and T, clipped Kramers opacity),
    a Dirichlet x_lo side, dt = 1e4 s; FP64, Jacobi-scaled stop at 1e-12 (the
    per-volume 1e-10 leaves ~2e-9 of error with this preconditioner)."""
    import numpy as np
    from oracle import fld_oracle as O
    a, b, c, d = nx0 // 4, 3 * nx0 // 4, ny0 // 4, 3 * ny0 // 4
    A, B, C, D = 2 * a, 2 * b, 2 * c, 2 * d
    qa, qb, qc, qd = A + (B - A) // 4, A + 3 * (B - A) // 4, C + (D - C) // 4, C + 3 * (D - C) // 4
    blocks = [(0, 0, 0, nx0, c), (0, 0, d, nx0, ny0 - d), (0, 0, c, a, d - c), (0, b, c, nx0 - b, d - c),
              (1, A, C, B - A, qc - C), (1, A, qd, B - A, D - qd), (1, A, qc, qa - A, qd - qc),
              (1, qb, qc, B - qb, qd - qc), (2, 2 * qa, 2 * qc, 2 * (qb - qa), 2 * (qd - qc))]
    bcs = [(1, 2e4), (0, 0.0), (0, 0.0), (0, 0.0)]
    fo = fld.Forest(blocks, nx0, ny0, 1e10, 1e10, bcs,
                    fld.default_options(precision="fp64", max_inner=20000, norm=1, rel_tol=1e-12))
    rng = np.random.default_rng(21)
    n = fo.cells
    rho = 1e-9 * np.exp(2.0 * rng.normal(size=n) * 0.5)
    T = 5e3 * np.exp(0.5 * rng.normal(size=n))
    kap = np.clip(1e22 * rho * T ** -3.5, 1e-4, 1e4)
    f = {"E": O.A_RAD * T ** 4, "T": T, "rho": rho, "kappa_R": kap, "kappa_P": kap.copy(), "c_v": np.full(n, 1e8)}
    t = {k: torch.tensor(v, dtype=torch.float64, device="cuda") for k, v in f.items()}
    E, Tg = t["E"].clone(), t["T"].clone()
    fo.step(E, Tg, t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], 1e4, check=False)  # warm-up
    ms = []
    for _ in range(3):
        E.copy_(t["E"])
        Tg.copy_(t["T"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = fo.step(E, Tg, t["rho"], t["kappa_R"], t["kappa_P"], t["c_v"], 1e4, check=False)
        torch.cuda.synchronize()
        ms.append(1e3 * (time.perf_counter() - t0))
    xc, yc, lv = fo.centres()
    fo.close()
    out = {"workload": f"block forest: {nx0}x{ny0} level-0 domain with nested level-1 and level-2 patches, "
                       f"{n} leaf cells, one matrix across levels; FP64 Jacobi-preconditioned CG",
           "cells": n, "ms_per_step": min(ms), "solves_per_s": 1e3 / min(ms), "inner_iters": info["inner_iters"],
           "rel_resid": info["rel_resid"], "status": info["status"],
           "mcell_iter_per_s": n * info["inner_iters"] / (min(ms) * 1e-3) / 1e6}
    if accuracy:
        from oracle import fld_forest as FF
        F = FF.build([FF.Block(*bk) for bk in blocks], 1e10, 1e10, nx0, ny0)
        ref = FF.step(F, f["E"], f["T"], f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], 1e4,
                      [O.BCSpec(k, v) for k, v in bcs])
        out["rel_l2_E"] = rel_l2(E.cpu().numpy(), ref.E)
        out["rel_l2_T"] = rel_l2(Tg.cpu().numpy(), ref.T)
    return out


def defaults(fld, **kw):
    return fld.default_options(**kw)


def options(fld, prec, tuned, norm=0):
    o = defaults(fld, precision=prec, norm=norm)
    if tuned is not None:
        for k in ("smoother", "mg_coarse_max", "mg_coarse_op", "chunk", "use_graph", "mg_cycle"):
            setattr(o, k, getattr(tuned, k))
    return o


def copy_calibration(torch):
    n = 512 * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": 4 * n, "launches": 5}), flush=True)


def main():
    global NO_GRAPH
    args = parse()
    NO_GRAPH = args.no_graph
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: this build has no multi-GPU path (the stress grid would shard "
                                   "into theta slabs, the batched blocks by count; see the design notes)"}),
              flush=True)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return
    import paper_2602_12545_amd as fld
    from paper_2602_12545_amd import tune as tuner
    import fld_workloads as W

    prob = W.make_c5()
    ncell = prob.nx * prob.ny
    f = dev_fields(torch, prob)
    prec = args.precision
    cyc, probe = pick_cycle(fld, torch, prob, f, prec, args.mg_cycle)
    ctx = make_ctx(fld, prob, stress_options(fld, prec, cyc))
    if args.warmup > 0:
        run_sequence(fld, torch, prob, f, None, args.warmup, ctx)
    sec, infos, _ = run_sequence(fld, torch, prob, f, None, args.steps, ctx)
    its = [i["inner_iters"] for i in infos]
    cname = {0: "V", 1: "K", 2: "W2", 3: "KL_K", 4: "KL_W2"}
    out = {
        "metric": METRIC,
        "value": 1.0 / sec,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "f32+f64", "fp64": "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": "c5: 4096x2048 spherical-polar stress recipe (lognormal kappa, contrast 1e8; "
                               "c_v=1e6, dt=1e5 s), consecutive implicit FLD steps through fld_steps (steps queued "
                               "back to back, CG iterations in captured two-slot chunks read one chunk behind "
                               "by the host), part of its 100-step sequence; one "
                               "benchmark step = one implicit step to 1e-10",
                   "cells": ncell, "precision": prec, "rel_tol": 1e-10, "norm": "Jacobi-scaled",
                   "mg_cycle": cname[cyc], "cycle_probe": probe,
                   "timed": f"one fld_steps call of {args.steps} steps from the initial state, after "
                            f"{args.warmup} warm-up steps"},
        "inner_iters": sum(its) / len(its),
        "iters": its,
        "mcell_iter_per_s": ncell * (sum(its) / len(its)) / sec / 1e6,
        "final_rel_resid": max(i["rel_resid"] for i in infos),
        "status": sorted(set(i["status"] for i in infos)),
    }
    if not args.no_profile:
        out["roofline"] = roofline(ctx)
    ctx.close()
    cycles = {prec: cyc}
    if not args.no_fp64 and prec != "fp64":
        # the same warm-up and timed steps in FP64, on FP64's own fastest cycle
        c64, probe64 = pick_cycle(fld, torch, prob, f, "fp64", args.mg_cycle)
        cycles["fp64"] = c64
        ctx = make_ctx(fld, prob, stress_options(fld, "fp64", c64))
        if args.warmup > 0:
            run_sequence(fld, torch, prob, f, None, args.warmup, ctx)
        sec64, inf64, _ = run_sequence(fld, torch, prob, f, None, args.steps, ctx)
        ctx.close()
        its64 = [i["inner_iters"] for i in inf64]
        out["fp64_same_steps"] = {"ms_per_step": sec64 * 1e3, "inner_iters": sum(its64) / len(its64),
                                  "iters": its64, "mg_cycle": cname[c64], "cycle_probe": probe64,
                                  "status": sorted(set(i["status"] for i in inf64))}
        out["mixed_vs_fp64"] = sec64 / sec
    if not args.no_sequence:
        seq = {"workload": f"the stress recipe's {SEQUENCE}-step sequence from its initial state, one fld_steps "
                           "call per precision, each on the fastest cycle of its probe"}
        ms, inf, _ = run_sequence(fld, torch, prob, f, stress_options(fld, prec, cyc), SEQUENCE)
        seq[prec] = summarise(prob, 1e3 * ms, inf)
        seq[prec]["mg_cycle"] = cname[cyc]
        if "fp64" in cycles and prec != "fp64":
            c64 = cycles["fp64"]
            ms, inf, _ = run_sequence(fld, torch, prob, f, stress_options(fld, "fp64", c64), SEQUENCE)
            seq["fp64"] = summarise(prob, 1e3 * ms, inf)
            seq["fp64"]["mg_cycle"] = cname[c64]
            seq["mixed_vs_fp64"] = seq["fp64"]["ms_per_step"] / seq[prec]["ms_per_step"]
        out["sequence_100"] = seq
    del f
    torch.cuda.empty_cache()
    if not args.no_accuracy:
        out["accuracy_stress_slab"] = stress_slab_accuracy(fld, torch, W, cycles)
    if not args.no_extra:
        out["workloads"] = other_workloads(fld, torch, W, tuner, not args.no_accuracy)
        out["batched_blocks"] = batch_extra(fld, torch, W, tuner)
        if not args.no_accuracy:
            out["batched_blocks"]["accuracy"] = batch_accuracy(fld, torch, W)
            out["batched_blocks"]["accuracy_stop_scaled_1e-12"] = batch_accuracy(fld, torch, W, 1, 1e-12)
        out["forest"] = forest_extra(fld, torch, not args.no_accuracy)
        out["substep"] = substep_extra(fld, torch, W, None)
        out["advection"] = advection_extra(fld, torch, W, None)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
