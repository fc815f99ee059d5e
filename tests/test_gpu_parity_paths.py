"""Bit-exact oracle parity on the paths the larger workloads take: the batched
kernel with many diagonal chunks (C3, C4, C5), three special primes and two
digits (C4), the grid partition case (Sec. 4.2, Table 3's last column), and
truncated samples of the full-size launch configurations (C3's 64-product
batch, the N = 2^15 job's m' = 2048 product).

Every oracle input is made by the oracle (integer plaintexts from its encoder
or its random integers, ciphertexts from its encryption with the shared
counter-based generator); the HIP path gets the same integers through the
C ABI (pvfl_pt_import, pvfl_encrypt_coeffs) and the output ciphertexts are
compared per coefficient-domain residue.

A truncated sample keeps the plaintexts of diagonals i < d and sets the rest
to zero.  The HIP path still runs the whole plan in its launch configuration
(every rotation key, every work item); a zero plaintext makes its term zero
in every residue, so the result equals the oracle's evaluation of the plan's
first d diagonals.  d is chosen to cross a chunk boundary of the fused kernel
and its re-centring points.  Needs an MI355X."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from oracle import plans as PL
from paper_2405_00482_amd import pvfl
from paper_2405_00482_amd import tune
from paper_2405_00482_amd import workloads as W

from gpu_util import context, dev_f64, dev_i64, export_ct, first_mismatch, torch

pytestmark = pytest.mark.gpu

WORKERS = max(1, min(16, os.cpu_count() or 1))
SEED_SK, SEED_KEYS, SEED_ENC = 21, 22, 23


def oracle_keys(prm, s, galois, seed):
    """the oracle's switching keys for every Galois element (independent, so threaded)"""
    from concurrent.futures import ThreadPoolExecutor
    gal = sorted(set(int(g) for g in galois))
    with ThreadPoolExecutor(WORKERS) as ex:
        return dict(zip(gal, ex.map(lambda g: O.rotkey_gen(prm, s, g, seed), gal)))


class Truncated:
    """a hybrid plan restricted to its diagonals i < d"""

    def __init__(self, plan, d):
        self.plan, self.d = plan, d

    def terms(self):
        return [t for t in self.plan.terms() if t[1] < self.d]


def hybrid_pt_ints_upto(prm, oplan, X, d):
    """the oracle's integer plaintexts of every diagonal, zero for i >= d"""
    out = []
    for b in range(oplan.row_blocks):
        for c in range(oplan.col_blocks):
            for i in range(oplan.mprime):
                if i < d:
                    out.append(O.encode(PL.hybrid_pt_slots(oplan, X, b, c, i), prm.N, prm.scale))
                else:
                    out.append(np.zeros(prm.N, dtype=np.int64))
    return out


def assert_cts_equal(got, want, what):
    for b, w in enumerate(want):
        for half, ref in ((0, w.c0), (1, w.c1)):
            mm = first_mismatch(got[b, half], np.asarray(ref, dtype=np.uint64))
            assert mm is None, f"{what} out {b}.{half}: first mismatch at {mm[0]} gpu={mm[1]} oracle={mm[2]} " \
                               f"({mm[3]} differ)"


class Product:
    """one X [[y]] product: the oracle's plan and inputs, and device buffers
    holding the same integers"""

    def __init__(self, prm, ctx, sk, s, plan, X, y, enc_seed, d=None):
        m, n = X.shape
        self.plan, self.X, self.y = plan, X, y
        self.oplan = PL.HybridPlan(m, n, prm.slots)
        info = plan.info
        assert info["mprime"] == self.oplan.mprime and info["n_pts"] == self.oplan.n_pts
        self.d = self.oplan.mprime if d is None else min(d, self.oplan.mprime)
        lv = prm.L
        N = prm.N
        self.pts = hybrid_pt_ints_upto(prm, self.oplan, X, self.d)
        cts_ints = PL.hybrid_ct_ints(prm, self.oplan, y, prm.scale)
        Q2 = 2 * (lv + 1) * N
        self.ct = dev_f64(plan.bytes("ct_in") // 8)
        self.octs = []
        for c, mi in enumerate(cts_ints):
            ctx.encrypt_coeffs(sk, lv, dev_i64(mi), enc_seed + c, self.ct[c * Q2:(c + 1) * Q2])
            self.octs.append(O.encrypt(prm, s, mi, lv, enc_seed + c))
        self.pt = dev_f64(plan.bytes("pt") // 8)
        self.import_pts(ctx, prm, self.pt)
        self.out = dev_f64(plan.bytes("ct_out") // 8)

    def import_pts(self, ctx, prm, pt):
        """the oracle's integers into a plaintext buffer of the plan (zero past d)"""
        K = self.plan.info["pt_limbs"]
        N = prm.N
        pt.zero_()
        # plaintext index (b * col_blocks + c) * m' + i: the first d of every block are nonzero
        blocks = self.oplan.row_blocks * self.oplan.col_blocks
        mp = self.oplan.mprime
        for blk in range(blocks):
            lo = blk * mp
            ints = np.stack(self.pts[lo:lo + self.d])
            ctx.pt_import(prm.L, K > prm.L + 1, dev_i64(ints), pt[lo * K * N:(lo + self.d) * K * N])

    def oracle(self, prm, okeys, lazy=True):
        plan = self.oplan if self.d == self.oplan.mprime else Truncated(self.oplan, self.d)
        return PL.hybrid_matmul(prm, plan, self.octs, self.pts, okeys, lazy, workers=WORKERS)

    def galois_used(self, N):
        return [O.galois_rotl(i, N) for i in range(1, self.d)]


def setup(name):
    prm = O.Params.from_dict(W.params_dict(name))
    ctx = context(name)
    sk = ctx.keygen(SEED_SK)
    s = O.keygen(prm, SEED_SK)
    return prm, ctx, sk, s


# ---------------------------------------------------------------------------
# the batched kernel over many diagonal chunks
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,shapes,group,chunk,vec", [
    # m' = 64 in 8 chunks (the partial-sum kernel's eight-loads loop) beside m' = 16
    ("C3", [(256, 2048), (64, 2048)], 2, 8, 2),
    # three special primes, two digits: m' = 64 in 16 and 22 chunks, m' = 8, m' = 1
    ("C4", [(300, 700), (40, 1000), (16, 256)], 2, 4, 2),
    ("C4", [(300, 700), (40, 1000), (16, 256)], 4, 3, 1),
    # ring 2^15 (split transforms): m' = 16 in 8 chunks beside a one-diagonal product
    ("C5", [(64, 4096), (3, 5)], 2, 2, 1),
    ("C5", [(64, 4096), (3, 5)], 2, 2, 2),
])
def test_batch_many_chunks_bit_exact(name, shapes, group, chunk, vec):
    prm, ctx, sk, s = setup(name)
    rng = np.random.default_rng(sum(m * n for m, n in shapes))
    plans = [ctx.plan(pvfl.PLAN_HYBRID, m, n, lazy=True) for (m, n) in shapes]
    prods = []
    for k, ((m, n), p) in enumerate(zip(shapes, plans)):
        X = rng.standard_normal((m, n))
        y = rng.uniform(-1, 1, n)
        prods.append(Product(prm, ctx, sk, s, p, X, y, SEED_ENC + 100 * k))
    assert max(-(-p.oplan.mprime // chunk) for p in prods) >= 8
    gal = sorted(set(g for p in plans for g in p.galois()))
    keys = ctx.rotkeys(sk, gal, SEED_KEYS)
    b = pvfl.Batch(ctx, plans, pt=[p.pt for p in prods], ct=[p.ct for p in prods], out=[p.out for p in prods],
                   keys=keys, group=group, chunk=chunk, vec=vec)
    b.matmul()
    torch().cuda.synchronize()
    okeys = oracle_keys(prm, s, gal, SEED_KEYS)
    for k, p in enumerate(prods):
        got = export_ct(ctx, prm.L, p.out, p.plan.info["ct_out"])
        assert_cts_equal(got, p.oracle(prm, okeys), f"{name} product {k} {shapes[k]} m'={p.oplan.mprime}")


# ---------------------------------------------------------------------------
# the grid partition case: m > N' and n > N' (Sec. 4.2; Table 3, last column)
# ---------------------------------------------------------------------------
def test_grid_partition_bit_exact_and_precise():
    """C1 (N' = 2048), X 4096 x 4096: 2 x 2 blocks of m' = 2048 diagonals, two
    input ciphertexts (column blocks, summed) and two outputs (row blocks).
    Random integer plaintexts check the wiring bit for bit; the real path then
    decrypts to X y within 2^-20."""
    prm, ctx, sk, s = setup("C1")
    N, lv = prm.N, prm.L
    m = n = 4096
    plan = ctx.plan(pvfl.PLAN_HYBRID, m, n, lazy=True)
    info = plan.info
    oplan = PL.HybridPlan(m, n, prm.slots)
    assert oplan.case == "grid"
    assert (info["row_blocks"], info["col_blocks"], info["mprime"]) == (2, 2, 2048)
    counts = oplan.op_counts()
    assert (info["n_mult"], info["n_add"], info["n_hstrot"], info["ct_in"], info["ct_out"]) == (
        counts["mult"], counts["add"], counts["hstrot"], 2, 2)
    rng = np.random.default_rng(4096)
    pts = [rng.integers(-(2 ** 30), 2 ** 30, size=N) for _ in range(oplan.n_pts)]
    cts_ints = [rng.integers(-(2 ** 30), 2 ** 30, size=N) for _ in range(oplan.col_blocks)]
    Q2 = 2 * (lv + 1) * N
    ct = dev_f64(plan.bytes("ct_in") // 8)
    octs = []
    for c, mi in enumerate(cts_ints):
        ctx.encrypt_coeffs(sk, lv, dev_i64(mi), SEED_ENC + c, ct[c * Q2:(c + 1) * Q2])
        octs.append(O.encrypt(prm, s, mi, lv, SEED_ENC + c))
    pt = dev_f64(plan.bytes("pt") // 8)
    ctx.pt_import(lv, True, dev_i64(np.stack(pts)), pt)
    gal = plan.galois()
    assert sorted(gal) == sorted(PL.hybrid_galois(oplan, N))
    keys = ctx.rotkeys(sk, gal, SEED_KEYS)
    out = dev_f64(plan.bytes("ct_out") // 8)
    plan.matmul(ct, pt, keys, out)
    got = export_ct(ctx, lv, out, 2)
    okeys = oracle_keys(prm, s, gal, SEED_KEYS)
    want = PL.hybrid_matmul(prm, oplan, octs, pts, okeys, True, workers=WORKERS)
    assert_cts_equal(got, want, "grid 4096x4096")
    # the real path on the GPU
    t = torch()
    f64 = dict(dtype=t.float64, device="cuda")
    X = rng.uniform(-1, 1, (m, n))
    y = rng.uniform(-1, 1, n)
    plan.encode_pt(t.from_numpy(X).to(**f64), pt)
    plan.encrypt(sk, t.from_numpy(y).to(**f64), SEED_ENC, ct)
    plan.matmul(ct, pt, keys, out)
    res = t.empty(m, **f64)
    plan.decrypt_decode(sk, out, res)
    ref = X @ y
    err = np.linalg.norm(res.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err < 2.0 ** -20, err


# ---------------------------------------------------------------------------
# three special primes, two digits (C4) in the per-call form
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lazy", [True, False])
def test_c4_hybrid_bit_exact(lazy):
    """C4 (6 + 3 primes, alpha = 3, beta = 2): a hybrid product with m' = 8
    (one ModUp, 7 hoisted rotations, lazy or per-rotation ModDown) and a
    row-partitioned one (m > N'), residue for residue"""
    prm, ctx, sk, s = setup("C4")
    rng = np.random.default_rng(44)
    for (m, n) in ((32, 2048), (16384, 4)):
        X = rng.uniform(-1, 1, (m, n))
        y = rng.uniform(-1, 1, n)
        plan = ctx.plan(pvfl.PLAN_HYBRID, m, n, lazy=lazy)
        p = Product(prm, ctx, sk, s, plan, X, y, SEED_ENC)
        gal = plan.galois()
        keys = ctx.rotkeys(sk, gal, SEED_KEYS)
        plan.matmul(p.ct, p.pt, keys, p.out)
        got = export_ct(ctx, prm.L, p.out, plan.info["ct_out"])
        okeys = oracle_keys(prm, s, gal, SEED_KEYS)
        want = PL.hybrid_matmul(prm, p.oplan, p.octs, p.pts, okeys, lazy)
        assert_cts_equal(got, want, f"C4 {m}x{n} {'lazy' if lazy else 'eager'}")
        zs = [O.decrypt_decode(prm, s, c, prm.scale ** 2) for c in want]
        res = PL.hybrid_lazy_ras(p.oplan, zs)
        assert np.linalg.norm(res - X @ y) / np.linalg.norm(X @ y) < 2.0 ** -20


# ---------------------------------------------------------------------------
# truncated samples of the full-size launch configurations
# ---------------------------------------------------------------------------
def test_c3_bench_configuration_truncated_sample():
    """C3's 64-product batch in the benchmark's launch options (tuner
    database): the two products of the first group (the largest m') carry the
    oracle's inputs with plaintexts zero past diagonal d = chunk + 9, so the
    sample crosses a chunk boundary and the re-centring after every eighth
    term; the two products with the fewest diagonals carry the oracle's full
    inputs.  The other 60 products run as in the benchmark."""
    prm, ctx, sk, s = setup("C3")
    N = prm.N
    shapes = W.c3_shapes(64)
    plans = [ctx.plan(pvfl.PLAN_HYBRID, m, n, lazy=True) for (m, n) in shapes]
    tuned = tune.lookup(tune.signature("C3", shapes))
    o = tuned["opts"] if tuned else {"group": 2, "chunk": 64, "vec": 2, "chunk_major": 1}
    gal = sorted(set(g for p in plans for g in p.galois()))
    keys = ctx.rotkeys(sk, gal, SEED_KEYS)
    mps = [p.info["mprime"] for p in plans]
    by_mp = sorted(range(64), key=lambda k: -mps[k])       # the batch groups products by m', descending
    big = by_mp[:o["group"]][:2]
    small = sorted(range(64), key=lambda k: mps[k])[:2]
    d = o["chunk"] + 9
    t = torch()
    f64 = dict(dtype=t.float64, device="cuda")
    prods = {}
    for k in big + small:
        XT, rk = W.c3_inputs(k, shapes[k])
        prods[k] = Product(prm, ctx, sk, s, plans[k], XT, rk, SEED_ENC + k, d=d if k in big else None)
    pt, ct, out = [], [], []
    for k, p in enumerate(plans):
        if k in prods:
            pt.append(prods[k].pt), ct.append(prods[k].ct), out.append(prods[k].out)
            continue
        XT, rk = W.c3_inputs(k, shapes[k])
        pt.append(t.empty(p.bytes("pt") // 8, **f64))
        p.encode_pt(t.from_numpy(XT).to(**f64), pt[-1])
        ct.append(t.empty(p.bytes("ct_in") // 8, **f64))
        p.encrypt(sk, t.from_numpy(rk).to(**f64), SEED_ENC + k, ct[-1])
        out.append(t.empty(p.bytes("ct_out") // 8, **f64))
    b = pvfl.Batch(ctx, plans, pt=pt, ct=ct, out=out, keys=keys, group=o["group"], chunk=o["chunk"], vec=o["vec"],
                   chunk_major=bool(o["chunk_major"]))
    b.matmul()
    t.cuda.synchronize()
    need = sorted(set(g for k in prods for g in prods[k].galois_used(N)))
    okeys = oracle_keys(prm, s, need, SEED_KEYS)
    for k, p in prods.items():
        got = export_ct(ctx, prm.L, p.out, 1)
        assert_cts_equal(got, p.oracle(prm, okeys), f"C3 product {k} {shapes[k]} m'={mps[k]} d={p.d}")


def test_c5_large_job_configuration_truncated_sample():
    """the N = 2^15 job: X^T (5000 x 4096) times two columns of [[R]] in the
    job's launch options (group 2, chunk 64, vec 2), one shared plaintext set
    (m' = 2048, 2047 rotation keys), plaintexts zero past diagonal 73"""
    prm, ctx, sk, s = setup("C5")
    N = prm.N
    XT, R = W.c5_inputs(cols=[0, 1])
    m, n = XT.shape
    plan = ctx.plan(pvfl.PLAN_HYBRID, m, n, lazy=True)
    assert plan.info["mprime"] == 2048
    d = 64 + 9
    cols = [Product(prm, ctx, sk, s, plan, XT, np.ascontiguousarray(R[:, c]), SEED_ENC + c, d=d) for c in range(2)]
    keys = ctx.rotkeys(sk, plan.galois(), SEED_KEYS)
    shared_pt = cols[0].pt
    del cols[1].pt
    b = pvfl.Batch(ctx, [plan, plan], pt=[shared_pt, shared_pt], ct=[c.ct for c in cols], out=[c.out for c in cols],
                   keys=keys, group=2, chunk=64, vec=2)
    b.matmul()
    torch().cuda.synchronize()
    okeys = oracle_keys(prm, s, cols[0].galois_used(N), SEED_KEYS)
    for c, p in enumerate(cols):
        got = export_ct(ctx, prm.L, p.out, 1)
        assert_cts_equal(got, p.oracle(prm, okeys), f"C5 column {c} d={d}")


# ---------------------------------------------------------------------------
# Alg. 3 at C4 in full, in the benchmark's launch configuration
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("part", ["forward", "backward"])
def test_c4_ctmat_full_size_bit_exact(part):
    """[[H]] (256 x 64) W (64 x 256) and the backward [[delta]] (256 x 256)
    W^T (256 x 64) at C4 (6 + 3 primes) with the widest column packing
    (pack 32), as the benchmark runs them: every output ciphertext bit-equal
    to the oracle's on every residue (Sec. 5.3, Alg. 3)."""
    from concurrent.futures import ThreadPoolExecutor
    prm, ctx, sk, s = setup("C4")
    N, lv = prm.N, prm.L
    H, Wm, delta = W.c4_inputs()
    A, B = (H, Wm) if part == "forward" else (delta, np.ascontiguousarray(Wm.T))
    m, n = A.shape
    nout = B.shape[1]
    pack = prm.slots // max(m, n)
    plan = ctx.plan(pvfl.PLAN_CTMAT, m, n, n_out=nout, pack=pack)
    oplan = PL.CtMatPlan(m, n, nout, prm.slots, pack)
    assert (plan.info["ct_in"], plan.info["ct_out"], plan.info["n_pts"]) == (oplan.ndiag, oplan.n_out_cts, oplan.n_pts)
    with ThreadPoolExecutor(WORKERS) as ex:
        msgs = list(ex.map(lambda i: O.encode(PL.ctmat_ct_slots(oplan, A, i), N, prm.scale), range(oplan.ndiag)))
        pts = list(ex.map(lambda ik: O.encode(PL.ctmat_pt_slots(oplan, B, ik[0], ik[1]), N, prm.scale),
                          [(i, k) for i in range(oplan.ndiag) for k in range(oplan.n_out_cts)]))
        octs = list(ex.map(lambda i: O.encrypt(prm, s, msgs[i], lv, SEED_ENC + i), range(oplan.ndiag)))
    Q = 2 * (lv + 1) * N
    ct = dev_f64(plan.bytes("ct_in") // 8)
    for i in range(oplan.ndiag):
        one = dev_f64(Q)
        ctx.encrypt_coeffs(sk, lv, dev_i64(msgs[i]), SEED_ENC + i, one)
        ct[i * Q:(i + 1) * Q] = one
    pt = dev_f64(plan.bytes("pt") // 8)
    ctx.pt_import(lv, False, dev_i64(np.stack(pts)), pt)
    out = dev_f64(plan.bytes("ct_out") // 8)
    plan.matmul(ct, pt, None, out)
    got = export_ct(ctx, lv, out, oplan.n_out_cts)
    assert_cts_equal(got, PL.ctmat_matmul(prm, oplan, octs, pts), f"C4 {part} [[{m}x{n}]] x {n}x{nout}, pack {pack}")
