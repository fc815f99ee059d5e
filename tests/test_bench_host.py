"""The benchmark's host-side pieces, on the CPU: the oracle tasks of the CPU
baseline (a whole C1 product, a C3 task over a diagonal range) and the
one-GPU contract of the command line."""
import subprocess
import sys

import pytest

import bench
from oracle import oracle as O
from oracle import plans as PL
from paper_2405_00482_amd import workloads as W


def test_cpu_hybrid_whole_c1_product():
    XT, r = W.c1_inputs()
    macs, t0, t1 = bench._cpu_hybrid("C1", XT, r, 0, 1 << 30, W.seeds("C1"), W.seeds("C1")["enc"])
    assert macs == XT.shape[0] * XT.shape[1] and t1 >= t0


def test_cpu_c3_task_credits_its_diagonal_share():
    shapes = W.c3_shapes(64)
    k = 0
    m, n = shapes[k]
    mp = PL.HybridPlan(m, n, O.Params.from_dict(W.params_dict("C3")).slots).mprime
    d1 = min(3, mp)
    macs, t0, t1 = bench._cpu_c3_range(k, shapes[k], 0, d1, W.seeds("C3"))
    assert macs == pytest.approx(m * n * d1 / mp) and t1 >= t0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr
