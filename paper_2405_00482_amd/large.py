"""The large configuration: X^T (5000 x 4096, 90% zeros, nonzeros N(0,1))
times [[R]] (4096 x 128, U[-1,1]) at N = 2^15 with 8 ciphertext primes and 2
special primes.  The 128 products X^T [[r_c]] share one hybrid plan (m' = 2048
diagonals per output ciphertext), one set of diagonal plaintexts and the 2047
rotation keys: the plaintexts are encoded once, the 128 input ciphertexts are
encrypted, multiplied in one batched launch (products grouped so that each key
and plaintext tile is streamed once per group), decrypted and read out.

Prints one JSON line: the job's cleartext MAC/s (5000 * 4096 * 128 per job,
inputs resident on the device, rotation keys generated beforehand), the time
of each phase (HIP events, median of the repeats) and the largest relative
error over the 128 columns.

    python -m paper_2405_00482_amd.large [--reps 3] [--chunk 64] [--group 2] [--vec 2]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--cols", type=int, default=128)
    ap.add_argument("--group", type=int, default=2)
    ap.add_argument("--chunk", type=int, default=64)
    ap.add_argument("--vec", type=int, default=2)
    a = ap.parse_args(argv)
    import torch
    from . import pvfl
    from . import workloads as W
    log = lambda s: print(s, file=sys.stderr, flush=True)  # noqa: E731
    name = "C5"
    seeds = W.seeds(name)
    XT, R = W.c5_inputs()
    R = np.ascontiguousarray(R[:, : a.cols])
    m, n = XT.shape
    ncol = R.shape[1]
    ctx = pvfl.Context.from_dict(W.params_dict(name), device=0)
    f64 = dict(dtype=torch.float64, device="cuda:0")
    plan = ctx.plan(pvfl.PLAN_HYBRID, m, n, lazy=True)
    info = plan.info
    log(f"[large] {m}x{n} times {n}x{ncol} at N=2^15: m'={info['mprime']}, {info['n_galois']} rotation keys")
    sk = ctx.keygen(seeds["sk"])
    t0 = time.perf_counter()
    keys = ctx.rotkeys(sk, plan.galois(), seeds["rotkeys"])
    torch.cuda.synchronize()
    log(f"[large] rotation keys generated in {time.perf_counter() - t0:.1f} s")
    Xd = torch.from_numpy(XT).to(**f64)
    cols = [torch.from_numpy(np.ascontiguousarray(R[:, c])).to(**f64) for c in range(ncol)]
    pt = torch.empty(plan.bytes("pt") // 8, **f64)
    cts = [torch.empty(plan.bytes("ct_in") // 8, **f64) for _ in range(ncol)]
    outs = [torch.empty(plan.bytes("ct_out") // 8, **f64) for _ in range(ncol)]
    ys = [torch.empty(m, **f64) for _ in range(ncol)]
    plans = [plan] * ncol
    b = pvfl.Batch(ctx, plans, X=None, v=cols, pt=[pt] * ncol, ct=cts, out=outs, y=ys, keys=keys,
                   group=a.group, chunk=a.chunk, vec=a.vec)
    info_b = b.info()
    log(f"[large] batch: {info_b['work_items']} work items, key stream {info_b['key_bytes'] / 2 ** 30:.1f} GiB")

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    phases = {"encode": [], "encrypt": [], "matmul": [], "decrypt": [], "job": []}
    for rep in range(a.reps + 1):
        e0 = ev()
        plan.encode_pt(Xd, pt)
        e1 = ev()
        b.encrypt(sk, seeds["enc"])
        e2 = ev()
        b.matmul()
        e3 = ev()
        b.decrypt(sk)
        e4 = ev()
        torch.cuda.synchronize()
        if rep == 0:
            continue  # warm-up
        for k, (x, y) in zip(("encode", "encrypt", "matmul", "decrypt", "job"),
                             ((e0, e1), (e1, e2), (e2, e3), (e3, e4), (e0, e4))):
            phases[k].append(x.elapsed_time(y))
        log(f"[large] rep {rep}: job {phases['job'][-1]:.2f} ms")
    ms = {k: float(np.median(v)) for k, v in phases.items()}
    ref = XT @ R
    got = np.stack([y.cpu().numpy() for y in ys], axis=1)
    errs = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
    macs = m * n * ncol
    out = {"workload": f"X^T ({m}x{n}, 90% zeros) times [[R]] ({n}x{ncol}), N=2^15, 8+2 primes, hybrid m'=2048, "
                       f"batched (group {a.group}, chunk {a.chunk}, vec {a.vec}), plaintexts shared",
           "macs_per_job": macs, "ms_per_job": ms["job"], "mac_per_s": macs / (ms["job"] * 1e-3),
           "phases_ms": ms, "max_rel_err": float(errs.max()), "key_stream_GiB": info_b["key_bytes"] / 2 ** 30}
    assert errs.max() < 2.0 ** -20, f"column error {errs.max()}"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    sys.exit(main())
