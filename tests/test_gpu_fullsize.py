"""The batched product at its full size and in the launch configuration the
benchmark times: 64 products at N = 2^14 with 4+1 primes, launch options from
the tuner database, replayed from a HIP graph.  Every product is checked
against the per-call form bit for bit, every decrypted result against X r
within 2^-20, and the two products with the fewest diagonals against the
oracle bit for bit (from the GPU's own integer plaintexts and input
ciphertexts, so the two FP64 encoders' rounding does not enter).  Needs an
MI355X."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import plans as PL
from paper_2405_00482_amd import pvfl
from paper_2405_00482_amd import tune
from paper_2405_00482_amd import workloads as W

from gpu_util import context, dev_u64, export, export_ct, first_mismatch, host_u64, torch

pytestmark = pytest.mark.gpu


def _centred_crt(r0, r1, q0, q1):
    """integers with residues r0 mod q0 and r1 mod q1, centred mod q0 q1"""
    r0 = r0.astype(object)
    r1 = r1.astype(object)
    t = ((r1 - r0) * pow(q0, -1, q1)) % q1
    x = r0 + q0 * t
    Q = q0 * q1
    return np.array([int(v - Q) if v > Q // 2 else int(v) for v in x], dtype=np.int64)


def test_c3_batch_full_size_bench_configuration():
    t = torch()
    name = "C3"
    prm = O.Params.from_dict(W.params_dict(name))
    ctx = context(name)
    N, lv = prm.N, prm.L
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
    # the oracle on the two products with the fewest diagonals
    s = O.keygen(prm, seeds["sk"])
    order = sorted(range(len(plans)), key=lambda k: plans[k].info["mprime"])[:2]
    for k in order:
        p = plans[k]
        m, n = shapes[k]
        info = p.info
        oplan = PL.HybridPlan(m, n, prm.slots)
        raw = export(ctx, lv, True, pt[k], info["n_pts"])           # [n_pts][K][N]
        pts = [_centred_crt(raw[i, 0], raw[i, 1], prm.q[0], prm.q[1]) for i in range(info["n_pts"])]
        cin = export_ct(ctx, lv, ct[k], info["ct_in"])
        octs = [O.Ciphertext(cin[c, 0], cin[c, 1], lv) for c in range(info["ct_in"])]
        okeys = {g: O.rotkey_gen(prm, s, g, seeds["rotkeys"]) for g in p.galois()}
        want = PL.hybrid_matmul(prm, oplan, octs, pts, okeys, True)
        got = export_ct(ctx, lv, out[k], info["ct_out"])
        for bo, w in enumerate(want):
            for half, ref in ((0, w.c0), (1, w.c1)):
                mm = first_mismatch(got[bo, half], np.asarray(ref, dtype=np.uint64))
                assert mm is None, f"product {k} ({m}x{n}, m'={info['mprime']}) out {bo}.{half}: {mm}"
