"""Benchmark of the packed-HE ciphertext x plaintext matrix product on one GPU.

Workload (default): 64 independent products X_k^T [[r_k]] at ring degree 2^14
with 4 ciphertext primes + 1 special prime, batch ~ logU[512, 4096] and
features ~ logU[32, 2000] (seeded), X ~ N(0,1), r ~ U[-1,1].  One step is the
whole path for all 64 products with inputs resident in HBM: plaintext packing
and encoding, encryption of r_k, the encrypted product, decryption + decoding +
lazy rotate-and-sum.  The metric is cleartext multiply-accumulates per second
(sum over products of m*n, unpadded) per wall second of the step.

Prints one JSON line.  --gpus > 1 is not supported (one process, one GPU).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP64 vector peak: 256 CUs x 64 FP64 FMA lanes per clock x 2 flops x 2.4 GHz
FP64_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
# the same units counted in operations: 256 CUs x 64 FP64 lanes x 2.4 GHz, every
# FP64 VALU instruction (multiply, add, round, FMA) one lane-operation
FP64_OP_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# timer class -> kernel symbol (template instances share the prefix)
KERNEL_SYMBOL = {"fused_diagonal": "k_diag_batch", "encode_pt": "k_encode_pt_batch", "modup": "k_modup",
                 "moddown": "k_moddown"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _cpu_sample(name, k, shape, n_diag, seeds):
    """One task of the CPU baseline: product k's first n_diag diagonals on the
    oracle, whole path (encode the plaintext diagonals, encode and encrypt r,
    the lazy-ModDown product, decrypt + decode + lazy RaS).  Rotation-key
    generation is set-up, done before the timer starts.  Returns the
    cleartext MACs covered (m n D / m') and the timed region's wall-clock
    start and end."""
    from paper_2405_00482_amd import workloads as W
    XT, r = W.c3_inputs(k, shape)
    return _cpu_hybrid(name, XT, r, 0, n_diag, seeds, seeds["enc"] + k)


def _cpu_c3_range(k, shape, d0, d1, seeds):
    """product k of the C3 batch, diagonals [d0, d1)"""
    from paper_2405_00482_amd import workloads as W
    XT, r = W.c3_inputs(k, shape)
    return _cpu_hybrid("C3", XT, r, d0, d1, seeds, seeds["enc"] + k)


def _cpu_hybrid(name, XT, r, d0, d1, seeds, enc_seed):
    """X^T [[r]] by the hybrid plan with lazy ModDown on the oracle, the terms
    of diagonals [d0, d1) (d1 capped at m'; all of them for [0, m')); see
    _cpu_sample.  The MACs credited are m n (d1 - d0) / m'."""
    from oracle import oracle as O
    from oracle import plans as PL
    from paper_2405_00482_amd import workloads as W
    prm = O.Params.from_dict(W.params_dict(name))
    m, n = XT.shape
    plan = PL.HybridPlan(m, n, prm.slots)
    d1 = min(d1, plan.mprime)

    class Trunc:
        def terms(self):
            return [t for t in plan.terms() if d0 <= t[1] < d1]

    s = O.keygen(prm, seeds["sk"])
    keys = {O.galois_rotl(i, prm.N): O.rotkey_gen(prm, s, O.galois_rotl(i, prm.N), seeds["rotkeys"])
            for i in range(max(d0, 1), d1)}
    t0 = time.time()
    pts = [O.encode(PL.hybrid_pt_slots(plan, XT, 0, 0, i), prm.N, prm.scale) if d0 <= i < d1 else None
           for i in range(d1)]
    ct = O.encrypt(prm, s, PL.hybrid_ct_ints(prm, plan, r, prm.scale)[0], prm.L, enc_seed)
    out = PL.hybrid_matmul(prm, Trunc(), [ct], pts, keys, True)[0]
    z = O.decrypt_decode(prm, s, out, prm.scale ** 2)
    PL.hybrid_lazy_ras(plan, [z])
    t1 = time.time()
    return m * n * (d1 - d0) / plan.mprime, t0, t1


def _cpu_worker_ready(_):
    """load the oracle in a pool worker before the timed tasks"""
    from oracle import oracle as O
    O.lib()
    return os.getpid()


def _host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def cpu_baseline(name, shapes, seeds, single_tasks=2, single_diag=16, pool_tasks=32, pool_diag=24,
                 max_workers=16) -> dict:
    """The CPU oracle as it stands (untuned), timed on the host's cores on a
    bounded sample of the step: the first diagonals of the first products.
    * single-thread: products 0..single_tasks-1, first single_diag diagonals
      each, one after the other in this process;
    * all cores: products 0..pool_tasks-1, first pool_diag diagonals each, over
      a process pool of min(max_workers, usable cores) workers; the rate is
      the MACs of every task over the span from the first task's start to the
      last one's end.
    Both rates are cleartext MAC/s of the sample; applied to the whole step
    they are a per-diagonal extrapolation (every diagonal of a product costs
    the oracle the same work)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    model, nproc, usable = _host_cpu()
    macs1, dt1 = 0.0, 0.0
    for k in range(min(single_tasks, len(shapes))):
        mk, t0, t1 = _cpu_sample(name, k, shapes[k], single_diag, seeds)
        macs1 += mk
        dt1 += t1 - t0
    workers = max(1, min(max_workers, usable))
    tasks = list(range(min(pool_tasks, len(shapes))))
    # spawned workers start from a fresh interpreter (no GPU state is inherited)
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        list(ex.map(_cpu_worker_ready, range(workers)))   # start and load every worker before timing
        res = list(ex.map(_cpu_sample, [name] * len(tasks), tasks, [shapes[k] for k in tasks],
                          [pool_diag] * len(tasks), [seeds] * len(tasks)))
    macs_all = sum(r[0] for r in res)
    span = max(r[2] for r in res) - min(r[1] for r in res)
    step_macs = sum(m * n for (m, n) in shapes)
    return {"value": macs_all / span, "unit": "MAC/s", "cores": workers, "kind": "oracle",
            "sample": f"first {pool_diag} diagonals of products 0-{len(tasks) - 1} (whole path, rotation keys "
                      f"generated beforehand) on {workers} worker processes: {macs_all:.3g} MACs, "
                      f"{100 * macs_all / step_macs:.1f}% of the step's, in {span:.1f} s; a per-diagonal "
                      f"extrapolation when applied to the whole step",
            "single_thread": {"value": macs1 / dt1, "unit": "MAC/s", "cores": 1,
                              "sample": f"first {single_diag} diagonals of products 0-{single_tasks - 1}: "
                                        f"{macs1:.3g} MACs in {dt1:.1f} s"},
            "macs_covered": macs_all, "fraction_of_step_macs": macs_all / step_macs,
            "cpu_model": model, "nproc": nproc, "usable_cpus": usable, "threads": workers}


def _cpu_ctmat(A, B, seeds):
    """[[A]] B by Alg. 3 on the oracle at C4 with the widest column packing,
    the evaluating party's work as ctmat_c4 times it: encode B's plaintexts
    and the product (A's diagonal ciphertexts are encrypted beforehand)."""
    from oracle import oracle as O
    from oracle import plans as PL
    from paper_2405_00482_amd import workloads as W
    prm = O.Params.from_dict(W.params_dict("C4"))
    m, n = A.shape
    nout = B.shape[1]
    pack = prm.slots // max(m, n)
    plan = PL.CtMatPlan(m, n, nout, prm.slots, pack)
    s = O.keygen(prm, seeds["sk"])
    cts = [O.encrypt(prm, s, O.encode(PL.ctmat_ct_slots(plan, A, i), prm.N, prm.scale), prm.L, seeds["enc"] + i)
           for i in range(plan.ndiag)]
    t0 = time.time()
    pts = [O.encode(PL.ctmat_pt_slots(plan, B, i, k), prm.N, prm.scale)
           for i in range(plan.ndiag) for k in range(plan.n_out_cts)]
    PL.ctmat_matmul(prm, plan, cts, pts)
    return m * n * nout, time.time() - t0, pack


def cpu_full(max_workers=16) -> dict:
    """The CPU oracle on whole configurations (not part of the default run):
    C1 and C2 (one X^T [[r]] product each, every diagonal) and C4 (Alg. 3
    forward and backward) on one thread; C3's 64 products, every diagonal,
    over a process pool (one product per task, largest first; the rate is
    all MACs over the span from the first task's start to the last one's
    end); C5 (N = 2^15) truncated to one column and its first 64 diagonals,
    labelled as such.  Rotation keys are generated before each timer starts."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    from paper_2405_00482_amd import workloads as W
    from oracle import plans as PL
    model, nproc, usable = _host_cpu()
    res = {"cpu_model": model, "nproc": nproc, "usable_cpus": usable}
    for name, (XT, r) in (("C1", W.c1_inputs()), ("C2", W.c2_inputs())):
        macs, t0, t1 = _cpu_hybrid(name, XT, r, 0, 1 << 30, W.seeds(name), W.seeds(name)["enc"])
        res[name] = {"shape": f"{XT.shape[0]}x{XT.shape[1]}", "macs": macs, "s": t1 - t0,
                     "mac_per_s": macs / (t1 - t0), "threads": 1, "kind": "full"}
        log(f"[cpu-full] {name}: {macs:.3g} MACs in {t1 - t0:.2f} s on 1 thread")
    H, Wm, delta = W.c4_inputs()
    for part, A, B in (("forward", H, Wm), ("backward", delta, np.ascontiguousarray(Wm.T))):
        macs, dt, pack = _cpu_ctmat(A, B, W.seeds("C4"))
        res[f"C4_{part}"] = {"shape": f"[[{A.shape[0]}x{A.shape[1]}]] x {B.shape[0]}x{B.shape[1]}", "pack": pack,
                             "macs": macs, "s": dt, "mac_per_s": macs / dt, "threads": 1, "kind": "full"}
        log(f"[cpu-full] C4 {part}: {macs:.3g} MACs in {dt:.2f} s on 1 thread")
    shapes = W.c3_shapes(64)
    seeds = W.seeds("C3")
    from oracle import oracle as O
    slots = O.Params.from_dict(W.params_dict("C3")).slots
    # tasks of at most 64 diagonals of one product, so that no product's
    # diagonals line up on one worker; each task encrypts r_k, accumulates its
    # diagonals, and ModDowns and decrypts its partial result
    tasks = []
    for k, sh in enumerate(shapes):
        mp_k = PL.HybridPlan(*sh, slots).mprime
        tasks += [(k, sh, d0, min(d0 + 64, mp_k)) for d0 in range(0, mp_k, 64)]
    workers = max(1, min(max_workers, usable))
    from concurrent.futures import as_completed
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        list(ex.map(_cpu_worker_ready, range(workers)))
        futs = [ex.submit(_cpu_c3_range, k, sh, d0, d1, seeds) for (k, sh, d0, d1) in tasks]
        out = []
        for f in as_completed(futs):
            out.append(f.result())
            if len(out) % 16 == 0:
                log(f"[cpu-full] C3: {len(out)}/{len(futs)} tasks done")
    macs = sum(o[0] for o in out)
    span = max(o[2] for o in out) - min(o[1] for o in out)
    res["C3"] = {"shape": f"64 products in {len(tasks)} tasks of at most 64 diagonals", "macs": macs, "s": span,
                 "mac_per_s": macs / span, "threads": workers, "kind": "full"}
    log(f"[cpu-full] C3: {macs:.3g} MACs in {span:.1f} s on {workers} processes")
    XT, R = W.c5_inputs(cols=[0])
    log("[cpu-full] C5 (truncated) ...")
    macs, t0, t1 = _cpu_hybrid("C5", XT, np.ascontiguousarray(R[:, 0]), 0, 64, W.seeds("C5"), W.seeds("C5")["enc"])
    res["C5"] = {"shape": f"{XT.shape[0]}x{XT.shape[1]} times one column, first 64 of 2048 diagonals",
                 "macs": macs, "s": t1 - t0, "mac_per_s": macs / (t1 - t0), "threads": 1,
                 "kind": "truncated (a per-diagonal extrapolation when applied to the whole job)"}
    log(f"[cpu-full] C5 (truncated): {macs:.3g} MACs in {t1 - t0:.2f} s on 1 thread")
    return res


def ctmat_c4(reps: int = 5) -> dict:
    """The encrypted-matrix operand form at its configuration (N = 2^14, 6+3
    primes): [[H]] (256 x 64) W (64 x 256), and the backward [[delta]] (256 x
    256) W^T, by Alg. 3 with the widest column packing (N/2 / max(m, n)).  Times
    the evaluating party's work per call -- encoding W and the product -- with
    HIP events (median of reps) and checks the decrypted product."""
    import torch
    from paper_2405_00482_amd import pvfl
    from paper_2405_00482_amd import workloads as W
    ctx = pvfl.Context.from_dict(W.params_dict("C4"), device=0)
    seeds = W.seeds("C4")
    sk = ctx.keygen(seeds["sk"])
    H, Wm, delta = W.c4_inputs()
    f64 = dict(dtype=torch.float64, device="cuda:0")
    out = {}
    for name, A, B in (("forward", H, Wm), ("backward", delta, np.ascontiguousarray(Wm.T))):
        m, n = A.shape
        nout = B.shape[1]
        pack = (ctx.N // 2) // max(m, n)
        plan = ctx.plan(pvfl.PLAN_CTMAT, m, n, n_out=nout, pack=pack)
        Bd = torch.from_numpy(B).to(**f64)
        pt = torch.empty(plan.bytes("pt") // 8, **f64)
        ct = torch.empty(plan.bytes("ct_in") // 8, **f64)
        o = torch.empty(plan.bytes("ct_out") // 8, **f64)
        y = torch.empty(m * nout, **f64)
        plan.encrypt(sk, torch.from_numpy(A).to(**f64), seeds["enc"], ct)
        ts = []
        for _ in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.encode_pt(Bd, pt)
            plan.matmul(ct, pt, None, o)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts[1:]))
        plan.decrypt_decode(sk, o, y)
        ref = A @ B
        err = float(np.linalg.norm(y.cpu().numpy().reshape(m, nout) - ref) / np.linalg.norm(ref))
        assert err < 2.0 ** -20, f"C4 {name}: decrypted product off by {err}"
        out[name] = {"shape": f"[[{m}x{n}]] x {n}x{nout}", "pack": pack, "ms": ms,
                     "mac_per_s": m * n * nout / (ms * 1e-3), "rel_err": err}
        log(f"[bench] C4 {name}: {m}x{n} times {n}x{nout}, pack {pack}: {ms:.3f} ms, "
            f"{m * n * nout / (ms * 1e-3):.3e} MAC/s, rel err 2^{np.log2(err):.1f}")
    return out


def ntt_throughput(ctx, level: int, polys: int = 1024, reps: int = 5) -> dict:
    """NTTs alone, both directions, on `polys` polynomials over every limb of
    Q u P at `level` (one limb transform per workgroup).  HIP events, median of
    reps.
    * forward: signed int64 coefficients imported into every limb (reduce,
      transform); algorithmic bytes = the int64 row once per polynomial plus
      8N written per limb, 8 N polys (1 + limbs);
    * inverse: the evaluation-domain limbs exported as canonical uint64
      coefficients; 8N read and 8N written per limb transform."""
    import torch
    N = ctx.N
    limbs = level + 1 + ctx.alpha
    g = torch.Generator(device="cuda:0").manual_seed(7)
    m = torch.randint(-(1 << 40), 1 << 40, (polys, N), dtype=torch.int64, device="cuda:0", generator=g)
    out = torch.empty(polys * limbs * N, dtype=torch.float64, device="cuda:0")
    back = torch.empty(polys * limbs * N, dtype=torch.int64, device="cuda:0")

    def median_ms(fn):
        ts = []
        for _ in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts[1:]))

    ms_f = median_ms(lambda: ctx.pt_import(level, True, m, out))
    ms_i = median_ms(lambda: ctx.export_coeffs(level, True, out, polys, back))
    res = {"limb_transforms": polys * limbs}
    for key, ms, nbytes in (("forward", ms_f, 8.0 * N * polys * (1 + limbs)), ("inverse", ms_i, 16.0 * N * polys * limbs)):
        gbps = nbytes / (ms * 1e-3) / 1e9
        res[key] = {"ms": ms, "bytes": nbytes, "algorithmic_GBps": gbps, "frac_of_hbm_peak": gbps / HBM_PEAK_GBS}
        log(f"[bench] NTT {key}: {polys * limbs} limb transforms at N={N} in {ms:.3f} ms, "
            f"{gbps:.1f} GB/s algorithmic ({gbps / HBM_PEAK_GBS:.2f} of HBM peak)")
    return res


def copy_calibration(nbytes=256 << 20, reps=3):
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "dispatches": reps}), flush=True)


def encode_flops(n_pts: int, pt_limbs: int, log_n: int) -> float:
    """Algorithmic FP64 operations of encoding n_pts plaintexts of pt_limbs
    limbs each at ring degree 2^log_n (an FMA counts two):
    * inverse canonical embedding: the M = N/2 point DFT of a real input, as
      an M/2-point complex FFT (5 (M/2) log2(M/2)) and the split into the
      M-point spectrum (9 M), plus the twist by the 2N-th roots (6 M) and the
      scaling and rounding of the N real coefficients (2 N);
    * per limb: reduction of each coefficient modulo q (4 N) and the
      negacyclic NTT, (N/2) log2 N butterflies of 10 operations each -- the
      modular product as an exact double-double product (mul + FMA), a
      quotient estimate (mul, round) and the remainder (FMA + add), then the
      butterfly's add and subtract."""
    N = 1 << log_n
    M = N // 2
    fft = 5 * (M // 2) * (log_n - 2) + 9 * M + 6 * M + 2 * N
    limb = 4 * N + 10 * (N // 2) * log_n
    return float(n_pts) * (fft + pt_limbs * limb)


def encode_ops(n_pts: int, pt_limbs: int, log_n: int) -> float:
    """Algorithmic FP64 operations of the same encoding, each FP64 instruction
    one operation (an FMA counts once): the canonical-embedding part as in
    encode_flops (it has no fused operations), and per limb the NTT's
    (N/2) log2 N butterflies at 8 (the modular product: multiply, FMA,
    multiply, round, FMA, add; then the butterfly's add and subtract) plus
    the re-centring of the half of the coefficients the first stage adds
    (multiply, round, FMA; the other half enter the modular product as they
    are).  This is the count the FP64 issue rate bounds."""
    N = 1 << log_n
    M = N // 2
    fft = 5 * (M // 2) * (log_n - 2) + 9 * M + 6 * M + 2 * N
    limb = 3 * (N // 2) + 8 * (N // 2) * log_n
    return float(n_pts) * (fft + pt_limbs * limb)


def measured_traffic(launch_key: str, kernel: str):
    """HBM bytes per dispatch from the committed counter summary, or None when
    the summary is missing, was taken for another launch configuration, or
    the kernel sources changed since."""
    from paper_2405_00482_amd.profile_summary import kernel_source_hash
    f = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "hbm_traffic_C3.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        rec = json.load(fh)
    if rec.get("workload") != launch_key or rec.get("source_hash") != kernel_source_hash():
        return None
    hits = [v for k, v in rec["kernels"].items() if k.split("<")[0] == kernel]
    if not hits:
        return None
    n = sum(v["dispatches"] for v in hits)
    return sum(v["traffic_bytes"] * v["dispatches"] for v in hits) / n


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--products", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c4", action="store_true", help="skip the encrypted-matrix (Alg. 3) measurement at C4")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--group", type=int, default=None, help="default: the tuner database's choice, else 2")
    ap.add_argument("--vec", type=int, default=None, help="default: the tuner database's choice, else 1")
    ap.add_argument("--chunk", type=int, default=None, help="default: the tuner database's choice, else 32")
    ap.add_argument("--chunk-major", type=int, default=None, help="default: the tuner database's choice, else 1")
    ap.add_argument("--percall-steps", type=int, default=2)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (for scaling the HBM byte counters)")
    ap.add_argument("--cpu-full", action="store_true",
                    help="only time the CPU oracle on whole configurations (C1-C4 in full, C5 truncated); "
                         "several minutes on 16 cores")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.cpu_full:
        print(json.dumps({"cpu_full": cpu_full()}), flush=True)
        return

    import torch
    from paper_2405_00482_amd import pvfl
    from paper_2405_00482_amd import workloads as W

    name = "C3"
    dev = "cuda:0"
    torch.cuda.set_device(0)
    seeds = W.seeds(name)
    d = W.params_dict(name)
    ctx = pvfl.Context.from_dict(d, device=0)
    shapes = W.c3_shapes(args.products)
    log(f"[bench] {name}: {len(shapes)} products, N=2^{d['logN']}, primes {len(d['q'])}+{len(d['p'])}")
    plans = [ctx.plan(pvfl.PLAN_HYBRID, m, n, lazy=True) for (m, n) in shapes]
    gal = sorted(set(g for p in plans for g in p.galois()))
    sk = ctx.keygen(seeds["sk"])
    t0 = time.perf_counter()
    keys = ctx.rotkeys(sk, gal, seeds["rotkeys"])
    log(f"[bench] {len(gal)} rotation keys generated in {time.perf_counter() - t0:.2f} s")
    f64 = dict(dtype=torch.float64, device=dev)
    Xs, rs, pts, cts, outs, ys = [], [], [], [], [], []
    for k, (m, n) in enumerate(shapes):
        XT, r = W.c3_inputs(k, (m, n))
        Xs.append(torch.from_numpy(XT).to(dev))
        rs.append(torch.from_numpy(r).to(dev))
        p = plans[k]
        pts.append(torch.empty(p.bytes("pt") // 8, **f64))
        cts.append(torch.empty(p.bytes("ct_in") // 8, **f64))
        outs.append(torch.empty(p.bytes("ct_out") // 8, **f64))
        ys.append(torch.empty(m, **f64))
    ws = torch.empty(max(p.bytes("workspace") for p in plans) // 8 + 1, **f64)
    macs = sum(m * n for (m, n) in shapes)
    pt_gib = sum(t.numel() for t in pts) * 8 / 2 ** 30
    log(f"[bench] {macs} cleartext MACs per step, {pt_gib:.2f} GiB of plaintexts")

    from paper_2405_00482_amd import tune
    tuned = tune.lookup(tune.signature(name, shapes))
    topts = tuned["opts"] if tuned else {"group": 2, "chunk": 32, "vec": 1, "chunk_major": 1}
    for k in ("group", "chunk", "vec", "chunk_major"):
        if getattr(args, k) is None:
            setattr(args, k, topts[k])
    from_db = tuned is not None and all(getattr(args, k) == topts[k]
                                       for k in ("group", "chunk", "vec", "chunk_major"))
    log(f"[bench] launch options group {args.group}, chunk {args.chunk}, vec {args.vec}, chunk_major "
        f"{args.chunk_major}{' (tuner database)' if from_db else ''}")
    batch = pvfl.Batch(ctx, plans, X=Xs, v=rs, pt=pts, ct=cts, out=outs, y=ys, keys=keys,
                       group=args.group, chunk=args.chunk, vec=args.vec, chunk_major=bool(args.chunk_major))
    binfo = batch.info()
    log(f"[bench] batch: {binfo['work_items']} work items, key stream {binfo['key_bytes'] / 2 ** 30:.2f} GiB, "
        f"plaintexts {binfo['pt_bytes'] / 2 ** 30:.2f} GiB")
    seed = seeds["enc"]

    def step_batched():
        batch.run(sk, seed, graph=not args.no_graph)

    def step_percall():
        for k, p in enumerate(plans):
            p.encode_pt(Xs[k], pts[k])
            p.encrypt(sk, rs[k], seed + k, cts[k])
            p.matmul(cts[k], pts[k], keys, outs[k], ws)
            p.decrypt_decode(sk, outs[k], ys[k])

    def timed(fn, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    for w in range(args.warmup):
        step_batched()
        torch.cuda.synchronize()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    ms_per_step = timed(step_batched, args.steps)
    log(f"[bench] batched{' (graph replay)' if not args.no_graph else ''}: {args.steps} steps, {ms_per_step:.3f} ms/step")
    # correctness of the timed outputs
    errs = []
    for k in range(len(plans)):
        got = ys[k].cpu().numpy()
        ref = Xs[k].cpu().numpy() @ rs[k].cpu().numpy()
        errs.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
    log(f"[bench] max relative error over products: 2^{np.log2(max(errs)):.2f}")
    assert max(errs) < 2.0 ** -20, "decrypted products miss the 2^-20 bound"

    # per-kernel HIP-event timing: the same batched step, launched eagerly
    ctx.timing_enable(True)
    for cls in range(4):
        ctx.timing_read(cls)
    ms_instrumented = timed(lambda: batch.run(sk, seed, graph=False), args.steps)
    ctx.timing_enable(False)
    log(f"[bench] batched, eager with kernel timers: {ms_instrumented:.3f} ms/step")
    classes = {pvfl.TIMING_DIAG: "fused_diagonal", pvfl.TIMING_ENCODE: "encode_pt",
               pvfl.TIMING_MODUP: "modup", pvfl.TIMING_MODDOWN: "moddown"}
    kt = {}
    for cls, nm in classes.items():
        tot_ms, n_launch, by = ctx.timing_read(cls)
        kt[nm] = {"ms_per_step": tot_ms / args.steps, "launches": n_launch, "bytes": by, "total_ms": tot_ms}
        log(f"[bench] {nm}: {tot_ms / args.steps:.3f} ms/step over {n_launch} launches, "
            f"{by / max(tot_ms, 1e-9) / 1e6:.1f} GB/s algorithmic")
    dom = max(kt, key=lambda k: kt[k]["total_ms"])
    dk = kt[dom]
    avg_launch_s = dk["total_ms"] * 1e-3 / max(dk["launches"], 1)
    extra = {}
    if dom == "encode_pt":
        # FP64-ALU bound (about 8 operations per HBM byte): algorithmic FP64
        # operations against the FP64 issue rate; the FLOP view beside it
        infos = [p.info for p in plans]
        ops = sum(encode_ops(i["n_pts"], i["pt_limbs"], d["logN"]) for i in infos)
        flops = sum(encode_flops(i["n_pts"], i["pt_limbs"], d["logN"]) for i in infos)
        bound, unit, peak, per_launch = "alu", "T FP64-op/s", FP64_OP_PEAK_TOPS, ops
        achieved = ops / avg_launch_s / 1e12
        extra = {"flops_per_launch": flops, "tflops": flops / avg_launch_s / 1e12,
                 "frac_of_fp64_flop_peak": flops / avg_launch_s / 1e12 / FP64_PEAK_TFLOPS}
    else:
        bound, unit, peak = "hbm", "GB/s", HBM_PEAK_GBS
        per_launch = dk["bytes"] / max(dk["launches"], 1)
        achieved = per_launch / avg_launch_s / 1e9
    launch_key = f"C3 x{len(shapes)}, group {args.group}, chunk {args.chunk}, vec {args.vec}" + \
        ("" if args.chunk_major else ", slot-major")
    traffic = measured_traffic(launch_key, KERNEL_SYMBOL[dom])
    # the key-switch kernel (fused diagonal: rotations' key inner products and the
    # plaintext products) against HBM, whichever kernel dominates
    kd = kt["fused_diagonal"]
    kd_s = kd["total_ms"] * 1e-3 / max(kd["launches"], 1)
    kd_bytes = kd["bytes"] / max(kd["launches"], 1)
    kd_traffic = measured_traffic(launch_key, KERNEL_SYMBOL["fused_diagonal"])
    # its arithmetic in FP64 operations (each instruction one): per (product,
    # rotated diagonal, limb, index) 2 beta key products and the 2 plaintext
    # products at 6 each (multiply, FMA, multiply, round, FMA, add), 2 (beta - 1)
    # + 2 additions, and P c0's addition on the Q limbs; diagonal 0 (no
    # rotation) only its 2 plaintext products and 2 additions
    lv1, alpha = len(d["q"]), len(d["p"])
    beta, K = -(-lv1 // alpha), lv1 + alpha
    elems = binfo["pt_bytes"] / 8
    elems0 = sum(p.info["row_blocks"] * p.info["col_blocks"] for p in plans) * K * ctx.N
    kd_ops = (elems - elems0) * (12 * beta + 12 + 2 * (beta - 1) + 2 + lv1 / K) + elems0 * (12 + 2)
    roofline_ks = {"bound": "hbm", "kernel": KERNEL_SYMBOL["fused_diagonal"],
                   "achieved": kd_bytes / kd_s / 1e9 if kd_s > 0 else 0.0, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": (kd_bytes / kd_s / 1e9 / HBM_PEAK_GBS) if kd_s > 0 else 0.0, "traffic": kd_traffic,
                   "bytes_per_launch": kd_bytes, "avg_launch_us": kd_s * 1e6,
                   "traffic_GBps": (kd_traffic / kd_s / 1e9) if (kd_traffic and kd_s > 0) else None,
                   "fp64_ops_per_launch": kd_ops,
                   "fp64_op_frac": (kd_ops / kd_s / 1e12 / FP64_OP_PEAK_TOPS) if kd_s > 0 else 0.0}
    ms_percall = None
    if args.percall_steps > 0:
        ms_percall = timed(step_percall, args.percall_steps)
        log(f"[bench] per-call form: {ms_percall:.3f} ms/step")

    result = {
        "metric": "encrypted MatMult cleartext MAC/s at N=2^14",
        "value": macs / (ms_per_step * 1e-3),
        "unit": "MAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"C3: {len(shapes)} products X^T[[r]], batch logU[512,4096], features logU[32,2000], "
                               f"N=2^14, 4+1 primes, Delta=2^40, hybrid plan, lazy ModDown, batched form "
                               f"(group {args.group}, chunk {args.chunk}, vec {args.vec}, chunk_major "
                               f"{args.chunk_major}{', autotuned' if from_db else ''})"
                               f"{'' if args.no_graph else ', HIP graph'}",
                   "macs_per_step": macs, "max_rel_err": max(errs),
                   "percall_ms_per_step": ms_percall, "instrumented_ms_per_step": ms_instrumented},
        "roofline": {"bound": bound, "kernel": KERNEL_SYMBOL[dom], "achieved": achieved, "peak": peak,
                     "unit": unit, "frac": achieved / peak, "traffic": traffic,
                     ("fp64_ops_per_launch" if bound == "alu" else "bytes_per_launch"): per_launch,
                     "hbm_bytes_per_launch": dk["bytes"] / max(dk["launches"], 1),
                     "avg_launch_us": avg_launch_s * 1e6, **extra},
        "roofline_keyswitch": roofline_ks,
        "ntt": ntt_throughput(ctx, len(d["q"]) - 1),
        "kernels": {k: {"ms_per_step": v["ms_per_step"], "launches_per_step": v["launches"] / args.steps,
                        "algorithmic_GBps": v["bytes"] / max(v["total_ms"] * 1e-3, 1e-12) / 1e9}
                    for k, v in kt.items()},
    }
    if not args.no_c4:
        result["c4_ctmat"] = ctmat_c4()
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        cb = cpu_baseline(name, shapes, seeds)
        result["cpu_baseline"] = cb
        log(f"[bench] cpu baseline: {cb['value']:.3e} MAC/s on {cb['cores']} processes "
            f"({100 * cb['fraction_of_step_macs']:.1f}% of the step's MACs), "
            f"{cb['single_thread']['value']:.3e} MAC/s single-threaded; {cb['cpu_model']}, nproc {cb['nproc']}")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
