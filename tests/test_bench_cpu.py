"""The benchmark's CPU leg on the host (no GPU): the oracle run on decoupled
theta slabs of a small stress grid in worker processes, with the fields the
benchmark line reports."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import fld_workloads as W  # noqa: E402


class _SmallStress:
    """The workload module's interface with the stress recipe shrunk to
    256 x 64 cells."""
    make_c5 = staticmethod(lambda: W.make_c5(nx=256, ny=64))
    theta_slab = staticmethod(W.theta_slab)
    make_c2 = staticmethod(W.make_c2)


def test_cpu_baseline_on_slabs():
    r = bench.cpu_baseline(_SmallStress, max_procs=2)
    assert r["kind"] == "oracle" and r["unit"] == "solves/s" and r["value"] > 0
    assert r["cores"] == min(2, len(os.sched_getaffinity(0))) and r["host_cores"] >= r["cores"]
    assert "256x64 grid cut into" in r["sample"] and "decoupled theta slabs" in r["sample"]


def test_slab_heights_text():
    assert bench.c5_rows([0, 128, 256]) == "128"
    assert bench.c5_rows([0, 100, 256]) == "100-156"
