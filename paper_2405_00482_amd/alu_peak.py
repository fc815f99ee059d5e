"""Arithmetic-throughput probe of the GPU: FP64 FMA, the binary64 modular
product the library uses (q < 2^48), the 64-bit-integer Shoup modular product
(q < 2^62), a bare 64 x 64 -> 128-bit integer product and a 32-bit integer
multiply-add, each as operations per second over the whole chip (HIP events,
median of repeats).  This is the measurement behind holding residues as
doubles rather than 64-bit integers.

    python -m paper_2405_00482_amd.alu_peak [--blocks 4096] [--iters 4096]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
PROBE_LIB = os.path.join(_HERE, "libpvfl_probe.so")
PROBES = {0: ("fp64_fma", 2), 1: ("fp64_mulmod_q48", 1), 2: ("u64_shoup_mulmod_q62", 1), 3: ("u64_mul128", 1),
          4: ("u32_mul_add", 1)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--blocks", type=int, default=4096)
    ap.add_argument("--iters", type=int, default=4096)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args(argv)
    import torch
    if not os.path.exists(PROBE_LIB):
        raise RuntimeError(f"{PROBE_LIB} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(PROBE_LIB)
    lib.pvfl_probe_alu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.pvfl_probe_alu.restype = ctypes.c_double
    out = torch.empty(a.blocks * 256, dtype=torch.int64, device="cuda:0")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    res = {}
    for probe, (name, flops_per_op) in PROBES.items():
        ts = []
        for _ in range(a.reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ops = lib.pvfl_probe_alu(probe, a.blocks, a.iters, ctypes.c_void_p(out.data_ptr()), stream)
            e1.record()
            torch.cuda.synchronize()
            if ops < 0:
                raise RuntimeError(f"probe {name} failed to launch")
            ts.append(e0.elapsed_time(e1))
        ms = sorted(ts[1:])[len(ts[1:]) // 2]
        res[name] = {"ops": ops, "ms": ms, "tera_ops_per_s": ops / (ms * 1e-3) / 1e12}
        print(f"[alu] {name}: {ops / (ms * 1e-3) / 1e12:.2f} T op/s ({ms:.3f} ms)", file=sys.stderr, flush=True)
    fma = res["fp64_fma"]["tera_ops_per_s"]
    res["fp64_fma"]["tflops"] = 2 * fma
    res["fp64_mulmod_over_u64_shoup"] = res["fp64_mulmod_q48"]["tera_ops_per_s"] / \
        res["u64_shoup_mulmod_q62"]["tera_ops_per_s"]
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    sys.exit(main())
