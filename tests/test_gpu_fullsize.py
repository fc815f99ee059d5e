"""The batched product at its full size and in the launch configuration the
benchmark times: 64 products at N = 2^14 with 4+1 primes, launch options from
the tuner database, replayed from a HIP graph.  Every product is checked
against the per-call form bit for bit and every decrypted result against X r
within 2^-20.  The oracle's residue-level check of this launch configuration,
on inputs the oracle makes, is test_gpu_parity_paths.py's truncated sample.
Needs an MI355X."""
import numpy as np
import pytest

from paper_2405_00482_amd import pvfl
from paper_2405_00482_amd import tune
from paper_2405_00482_amd import workloads as W

from gpu_util import context, torch

pytestmark = pytest.mark.gpu


def test_c3_batch_full_size_bench_configuration():
    t = torch()
    name = "C3"
    ctx = context(name)
    seeds = W.seeds(name)
    shapes = W.c3_shapes(64)
    plans = [ctx.plan(pvfl.PLAN_HYBRID, m, n, lazy=True) for (m, n) in shapes]
    gal = sorted(set(g for p in plans for g in p.galois()))
    sk = ctx.keygen(seeds["sk"])
    keys = ctx.rotkeys(sk, gal, seeds["rotkeys"])
    tuned = tune.lookup(tune.signature(name, shapes))
    o = tuned["opts"] if tuned else {"group": 2, "chunk": 32, "vec": 2, "chunk_major": 1}
    f64 = dict(dtype=t.float64, device="cuda")
    X, r = [], []
    for k, (m, n) in enumerate(shapes):
        XT, rk = W.c3_inputs(k, (m, n))
        X.append(t.from_numpy(XT).cuda())
        r.append(t.from_numpy(rk).cuda())

    def bufs():
        return ([t.zeros(p.bytes("pt") // 8, **f64) for p in plans], [t.zeros(p.bytes("ct_in") // 8, **f64) for p in plans],
                [t.zeros(p.bytes("ct_out") // 8, **f64) for p in plans], [t.zeros(m, **f64) for (m, n) in shapes])

    pt, ct, out, y = bufs()
    b = pvfl.Batch(ctx, plans, X=X, v=r, pt=pt, ct=ct, out=out, y=y, keys=keys, group=o["group"], chunk=o["chunk"],
                   vec=o["vec"], chunk_major=bool(o["chunk_major"]))
    for _ in range(2):                        # capture and first replay, then a second replay
        b.run(sk, seeds["enc"], graph=True)
    t.cuda.synchronize()
    # the per-call form, product by product
    pt2, ct2, out2, y2 = bufs()
    for k, p in enumerate(plans):
        p.encode_pt(X[k], pt2[k])
        p.encrypt(sk, r[k], seeds["enc"] + k, ct2[k])
        p.matmul(ct2[k], pt2[k], keys, out2[k])
        p.decrypt_decode(sk, out2[k], y2[k])
    t.cuda.synchronize()
    for k in range(len(plans)):
        for what, a, c in (("plaintexts", pt, pt2), ("ciphertexts", ct, ct2), ("products", out, out2),
                           ("results", y, y2)):
            assert t.equal(a[k], c[k]), f"product {k}: batched {what} differ from the per-call form"
        ref = X[k].cpu().numpy() @ r[k].cpu().numpy()
        err = np.linalg.norm(y[k].cpu().numpy() - ref) / np.linalg.norm(ref)
        assert err < 2.0 ** -20, f"product {k}: relative error {err}"
