"""Host-side checks of bench.py (CPU): the one-GPU contract, the FLOP model
it reports the roofline with, and the guard on the recorded traffic."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"] and "--gpus 2" in msg["error"]


def test_flop_model_per_step_and_polish():
    # F(m) = 28 (m(m+1) - 2) + 11 (m - 1) + 4 m
    for m in range(2, 7):
        assert bench.F_LEVEL[m] == 28 * (m * (m + 1) - 2) + 11 * (m - 1) + 4 * m
    # polish: d steps of (16 d + 13) FLOPs per root
    assert bench.polish_flops(6, 2) == 1308
    # one step at every level, one polynomial: sum of F(m) + shift, plus the start
    it = np.ones((5, 1), dtype=np.int32)
    assert bench.algorithmic_flops(it) == sum(bench.F_LEVEL.values()) + 5 * bench.F_WILKINSON \
        + bench.F_START
    assert bench.algorithmic_flops(it, shift=0, start=0) == sum(bench.F_LEVEL.values())


def test_lockstep_work_bounds_the_useful_work():
    rng = np.random.default_rng(0)
    it = rng.integers(0, 12, size=(5, 64 * 20)).astype(np.int32)
    useful = bench.algorithmic_flops(it, start=0)
    executed = bench.lockstep_flops(it)
    assert executed >= useful
    # equal counts within every wave: nothing is wasted
    same = np.repeat(rng.integers(0, 12, size=(5, 20)), 64, axis=1).astype(np.int32)
    assert bench.lockstep_flops(same) == bench.algorithmic_flops(same, start=0)


def test_traffic_record_only_for_the_profiled_kernel_and_workload():
    assert bench.measured_traffic("fp64", 4096) is None
    assert bench.measured_traffic("fp32_polish", 2048) is None
    t = bench.measured_traffic("fp32_polish", 4096)
    # either the record matches the built kernel (a plausible byte count) or
    # the kernel changed since it was taken / nothing is built (None)
    assert t is None or 3e9 < t < 2e10


def test_cpu_baseline_reports_all_cores_and_one_thread():
    import workloads
    a = workloads.gaussian(20000, seed=3)
    r, roots, n = bench.cpu_baseline(a, target_s=0.2)
    assert r["kind"] == "oracle" and r["unit"] == "polys/s" and r["value"] > 0
    assert roots.shape == (6, n) and 0 < n <= a.shape[1]
    one = r["single_thread"]
    assert one["cores"] == 1 and one["value"] > 0
    assert r["nproc"] >= 1 and r["host_cpu"]
