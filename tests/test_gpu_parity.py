"""Bit-exact parity of the HIP path (called through the C ABI) against the CPU
oracle, on coefficient-domain residues.  Needs an MI355X."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import plans as PL
from paper_2405_00482_amd import pvfl
from paper_2405_00482_amd import workloads as W

from gpu_util import context, dev_f64, dev_i64, dev_u64, export, export_ct, first_mismatch, host_u64

pytestmark = pytest.mark.gpu

SEED_SK, SEED_KEYS, SEED_ENC = 11, 12, 13


@pytest.fixture(scope="module", params=["C1", "C4", "C5"])
def c1(request):
    """a ring-2^12 parameter set; ring 2^14 with three special primes and two
    digits (C4); ring 2^15, whose limbs exceed LDS and take the split
    transform"""
    prm = O.Params.from_dict(W.params_dict(request.param))
    ctx = context(request.param)
    sk_gpu = ctx.keygen(SEED_SK)
    s = O.keygen(prm, SEED_SK)
    return prm, ctx, sk_gpu, s


def assert_same(got, want, what):
    mm = first_mismatch(np.asarray(got, dtype=np.uint64), np.asarray(want, dtype=np.uint64))
    assert mm is None, f"{what}: first mismatch at {mm[0]} gpu={mm[1]} oracle={mm[2]} ({mm[3]} differ)"


def test_import_export_roundtrip(c1):
    prm, ctx, _, _ = c1
    rng = np.random.default_rng(0)
    m = rng.integers(-(2 ** 62), 2 ** 62, size=(3, prm.N), dtype=np.int64)
    m[0, :4] = [0, -1, 2 ** 62, -(2 ** 62)]
    lv = prm.L
    pt = dev_f64(3 * (lv + 1 + prm.alpha) * prm.N)
    ctx.pt_import(lv, True, dev_i64(m), pt)
    got = export(ctx, lv, True, pt, 3)
    primes = prm.qp(lv)
    want = np.stack([np.stack([O.poly_from_signed(m[c], q) for q in primes]) for c in range(3)])
    assert_same(got, want, "import/export")


def test_secret_key_matches_oracle(c1):
    prm, ctx, sk_gpu, s = c1
    nl = prm.L + 1 + prm.alpha
    out = dev_u64(nl * prm.N)
    sk_gpu.export(out)
    got = host_u64(out).reshape(nl, prm.N)
    want = np.stack([O.poly_from_signed(s, q) for q in prm.qp(prm.L)])
    assert_same(got, want, "secret key")


def _encrypt_both(prm, ctx, sk_gpu, s, m, seed, level=None):
    lv = prm.L if level is None else level
    ct = dev_f64(2 * (lv + 1) * prm.N)
    ctx.encrypt_coeffs(sk_gpu, lv, dev_i64(m), seed, ct)
    return ct, O.encrypt(prm, s, m, lv, seed)


def test_encrypt_decrypt_match_oracle(c1):
    prm, ctx, sk_gpu, s = c1
    rng = np.random.default_rng(1)
    m = rng.integers(-(2 ** 40), 2 ** 40, size=prm.N)
    ct, oct_ = _encrypt_both(prm, ctx, sk_gpu, s, m, SEED_ENC)
    got = export_ct(ctx, prm.L, ct)[0]
    assert_same(got[0], oct_.c0, "c0")
    assert_same(got[1], oct_.c1, "c1")
    out = dev_u64((prm.L + 1) * prm.N)
    ctx.decrypt_coeffs(sk_gpu, prm.L, ct, out)
    assert_same(host_u64(out).reshape(prm.L + 1, prm.N), O.decrypt(prm, s, oct_), "decrypt")


def test_ct_times_pt_matches_oracle(c1):
    prm, ctx, sk_gpu, s = c1
    rng = np.random.default_rng(2)
    m = rng.integers(-(2 ** 30), 2 ** 30, size=prm.N)
    p = rng.integers(-(2 ** 30), 2 ** 30, size=prm.N)
    ct, oct_ = _encrypt_both(prm, ctx, sk_gpu, s, m, 21)
    lv = prm.L
    pt = dev_f64((lv + 1) * prm.N)
    ctx.pt_import(lv, False, dev_i64(p[None, :]), pt)
    out = dev_f64(2 * (lv + 1) * prm.N)
    ctx.ct_mul_pt(lv, ct, pt, out)
    want = O.ct_mul_pt(prm, oct_, O.reduce_signed(p, prm.q))
    got = export_ct(ctx, lv, out)[0]
    assert_same(got[0], want.c0, "ct*pt c0")
    assert_same(got[1], want.c1, "ct*pt c1")


def test_rotation_keys_match_oracle(c1):
    prm, ctx, sk_gpu, s = c1
    gal = [O.galois_rotl(1, prm.N), O.galois_rotr(3, prm.N)]
    keys = ctx.rotkeys(sk_gpu, gal, SEED_KEYS)
    nl = prm.L + 1 + prm.alpha
    bL = prm.beta(prm.L)
    for k, g in enumerate(keys.galois):
        out = dev_u64(bL * 2 * nl * prm.N)
        keys.export(k, out)
        got = host_u64(out).reshape(bL, 2, nl, prm.N)
        ok = O.rotkey_gen(prm, s, g, SEED_KEYS)
        for j in range(bL):
            assert_same(got[j, 0], ok.b[j], f"key g={g} b_{j}")
            assert_same(got[j, 1], ok.a[j], f"key g={g} a_{j}")


@pytest.mark.parametrize("hoisted", [False, True])
def test_rotation_matches_oracle(c1, hoisted):
    prm, ctx, sk_gpu, s = c1
    rng = np.random.default_rng(3)
    m = rng.integers(-(2 ** 35), 2 ** 35, size=prm.N)
    ct, oct_ = _encrypt_both(prm, ctx, sk_gpu, s, m, 31)
    for r in (1, 5):
        g = O.galois_rotl(r, prm.N)
        keys = ctx.rotkeys(sk_gpu, [g], SEED_KEYS)
        okey = O.rotkey_gen(prm, s, g, SEED_KEYS)
        out = dev_f64(2 * (prm.L + 1) * prm.N)
        ctx.rotate(keys, prm.L, ct, g, hoisted, out)
        if hoisted:
            want = O.hoisted_rotate(prm, oct_, O.modup(prm, prm.L, oct_.c1), okey)
        else:
            want = O.rotate(prm, oct_, okey)
        got = export_ct(ctx, prm.L, out)[0]
        assert_same(got[0], want.c0, f"rot {r} c0")
        assert_same(got[1], want.c1, f"rot {r} c1")


def test_rescale_matches_oracle(c1):
    prm, ctx, sk_gpu, s = c1
    rng = np.random.default_rng(4)
    m = rng.integers(-(2 ** 60), 2 ** 60, size=prm.N)
    ct, oct_ = _encrypt_both(prm, ctx, sk_gpu, s, m, 41)
    out = dev_f64(2 * prm.L * prm.N)
    ctx.rescale(prm.L, ct, out)
    want = O.rescale(prm, oct_)
    got = export_ct(ctx, prm.L - 1, out)[0]
    assert_same(got[0], want.c0, "rescale c0")
    assert_same(got[1], want.c1, "rescale c1")


# ---------------------------------------------------------------------------
# the matrix product
# ---------------------------------------------------------------------------
def run_hybrid_both(name, X, y, lazy, kind="hybrid", bsgs=0, hoisted=True):
    prm = O.Params.from_dict(W.params_dict(name))
    ctx = context(name)
    N = prm.N
    m, n = X.shape
    sk_gpu = ctx.keygen(SEED_SK)
    s = O.keygen(prm, SEED_SK)
    if kind == "hybrid":
        plan = ctx.plan(0, m, n, lazy=lazy, bsgs=bsgs, unhoisted=not hoisted)
        oplan = PL.HybridPlan(m, n, prm.slots)
        pts = (PL.bsgs_pt_ints(prm, oplan, X, prm.scale, bsgs) if bsgs
               else PL.hybrid_pt_ints(prm, oplan, X, prm.scale))
        cts_ints = PL.hybrid_ct_ints(prm, oplan, y, prm.scale)
    else:
        plan = ctx.plan(1, m, n, lazy=lazy, ras_in_ct=(kind == "diag_rot"), unhoisted=not hoisted)
        oplan = PL.DiagPlan(m, n, prm.slots, "rot" if kind == "diag_rot" else "lazy")
        pts = [O.encode(PL.diag_pt_slots(oplan, X, i), N, prm.scale) for i in range(oplan.ndiag)]
        cts_ints = [O.encode(PL.diag_ct_slots(oplan, y), N, prm.scale)]
    info = plan.info
    assert info["n_pts"] == len(pts)
    lv = prm.L
    gal = plan.galois()
    keys = ctx.rotkeys(sk_gpu, gal, SEED_KEYS)
    okeys = {g: O.rotkey_gen(prm, s, g, SEED_KEYS) for g in gal}
    # ciphertexts
    ct = dev_f64(plan.bytes("ct_in") // 8)
    octs = []
    for c, mi in enumerate(cts_ints):
        one = dev_f64(2 * (lv + 1) * N)
        ctx.encrypt_coeffs(sk_gpu, lv, dev_i64(mi), SEED_ENC + c, one)
        ct[c * 2 * (lv + 1) * N:(c + 1) * 2 * (lv + 1) * N] = one
        octs.append(O.encrypt(prm, s, mi, lv, SEED_ENC + c))
    pt = dev_f64(plan.bytes("pt") // 8)
    ctx.pt_import(lv, info["pt_limbs"] > lv + 1, dev_i64(np.stack(pts)), pt)
    out = dev_f64(plan.bytes("ct_out") // 8)
    plan.matmul(ct, pt, keys, out)
    got = export_ct(ctx, lv, out, info["ct_out"])
    if kind == "hybrid" and bsgs:
        want = PL.hybrid_matmul_bsgs(prm, oplan, octs, pts, okeys, bsgs)
    elif kind == "hybrid":
        want = PL.hybrid_matmul(prm, oplan, octs, pts, okeys, lazy, hoisted)
    else:
        want = [PL.diag_matmul(prm, oplan, octs[0], pts, okeys, lazy, hoisted)]
    for b, w in enumerate(want):
        assert_same(got[b, 0], w.c0, f"out {b} c0")
        assert_same(got[b, 1], w.c1, f"out {b} c1")
    return prm, s, want, oplan


@pytest.mark.parametrize("lazy", [True, False])
def test_hybrid_c1_bit_exact_and_precise(lazy):
    XT, r = W.c1_inputs()
    prm, s, outs, oplan = run_hybrid_both("C1", XT, r, lazy)
    z = O.decrypt_decode(prm, s, outs[0], prm.scale ** 2)
    got = PL.hybrid_lazy_ras(oplan, [z])
    err = np.linalg.norm(got - XT @ r) / np.linalg.norm(XT @ r)
    assert err < (2.0 ** -20 if lazy else 2.0 ** -18)


@pytest.mark.parametrize("lazy", [True, False])
def test_hybrid_c2_full_size_bit_exact_and_precise(lazy):
    """C2's own product, X^T (256 x 1024) [[r]] at N = 2^13 (m' = 64, 63
    hoisted rotations), with lazy and with eager ModDown"""
    XT, r = W.c2_inputs()
    prm, s, outs, oplan = run_hybrid_both("C2", XT, r, lazy)
    assert oplan.mprime == 64
    z = O.decrypt_decode(prm, s, outs[0], prm.scale ** 2)
    got = PL.hybrid_lazy_ras(oplan, [z])
    err = np.linalg.norm(got - XT @ r) / np.linalg.norm(XT @ r)
    assert err < (2.0 ** -20 if lazy else 2.0 ** -18)


@pytest.mark.parametrize("m,n", [(4096, 4), (4, 4096), (100, 37), (1, 1)])
def test_hybrid_partition_and_ragged(m, n):
    rng = np.random.default_rng(m + n)
    X = rng.uniform(-1, 1, (m, n))
    y = rng.uniform(-1, 1, n)
    run_hybrid_both("C1", X, y, True)


@pytest.mark.parametrize("name,m,n,lazy", [("C5", 16, 4096, True), ("C5", 16, 4096, False), ("C5", 3, 5, True)])
def test_hybrid_ring_2_15_bit_exact(name, m, n, lazy):
    """hybrid product at N = 2^15 (10 limbs over Q u P, 4 digits): residues equal the oracle's"""
    rng = np.random.default_rng(m + n)
    X = rng.uniform(-1, 1, (m, n))
    y = rng.uniform(-1, 1, n)
    prm, s, outs, oplan = run_hybrid_both(name, X, y, lazy)
    z = O.decrypt_decode(prm, s, outs[0], prm.scale ** 2)
    got = PL.hybrid_lazy_ras(oplan, [z])
    assert np.linalg.norm(got - X @ y) / np.linalg.norm(X @ y) < 2.0 ** -20


@pytest.mark.parametrize("m,n,bs", [(64, 256, 2), (64, 256, 4), (100, 37, 2), (4096, 64, 8), (64, 4096, 4)])
def test_bsgs_bit_exact(m, n, bs):
    """baby-step/giant-step schedule: residues equal the oracle's, including
    row and column partitions (several giant-step sums per output)"""
    rng = np.random.default_rng(m * 7 + n)
    X = rng.uniform(-1, 1, (m, n))
    y = rng.uniform(-1, 1, n)
    prm, s, outs, oplan = run_hybrid_both("C1", X, y, True, bsgs=bs)
    zs = [O.decrypt_decode(prm, s, ct, prm.scale ** 2) for ct in outs]
    got = PL.hybrid_lazy_ras(oplan, zs)
    assert np.linalg.norm(got - X @ y) / np.linalg.norm(X @ y) < 2.0 ** -20


def test_bsgs_rejects_bad_baby_steps():
    ctx = context("C1")
    for bs in (3, 1, 8):            # not a power of two; too small; m' = 8 needs bs <= 4
        with pytest.raises(pvfl.PvflError):
            ctx.plan(0, 64, 256, lazy=True, bsgs=bs)
    with pytest.raises(pvfl.PvflError):
        ctx.plan(0, 64, 256, lazy=False, bsgs=2)
    with pytest.raises(pvfl.PvflError):
        ctx.plan(1, 64, 16, lazy=True, bsgs=2)


@pytest.mark.parametrize("kind,m,n", [("hybrid", 16, 256), ("hybrid", 100, 37), ("hybrid", 4096, 4), ("hybrid", 4, 4096),
                                      ("diag", 64, 16), ("diag_rot", 16, 64)])
def test_unhoisted_bit_exact(kind, m, n):
    """every rotation a complete O3 rotation (Sec. 2; GALA's cost profile in
    Table 2): residues equal the oracle's, counts are Table 2's GALA row"""
    rng = np.random.default_rng(m * 3 + n)
    X = rng.uniform(-1, 1, (m, n))
    y = rng.uniform(-1, 1, n)
    prm, s, outs, oplan = run_hybrid_both("C1", X, y, lazy=False, kind=kind, hoisted=False)
    ctx = context("C1")
    if kind == "hybrid":
        info = ctx.plan(0, m, n, lazy=False, unhoisted=True).info
        want = oplan.op_counts(unhoisted=True)
        assert (info["n_rot"], info["n_hstrot"], info["n_mult"]) == (want["rot"], want["hstrot"], want["mult"])
        zs = [O.decrypt_decode(prm, s, ct, prm.scale ** 2) for ct in outs]
        got = PL.hybrid_lazy_ras(oplan, zs)
        assert np.linalg.norm(got - X @ y) / np.linalg.norm(X @ y) < 2.0 ** -18


def test_unhoisted_rejects_other_schedules():
    ctx = context("C1")
    with pytest.raises(pvfl.PvflError):
        ctx.plan(0, 64, 256, lazy=True, unhoisted=True)       # O3 rotations are finished one by one
    with pytest.raises(pvfl.PvflError):
        ctx.plan(2, 16, 64, lazy=False, unhoisted=True)       # ROW has its own rotations
    with pytest.raises(pvfl.PvflError):
        ctx.plan(3, 16, 64, n_out=4, lazy=False, unhoisted=True)


@pytest.mark.parametrize("kind,m,n", [("diag", 64, 16), ("diag", 16, 64), ("diag_rot", 16, 64)])
def test_diag_plan_bit_exact(kind, m, n):
    rng = np.random.default_rng(7)
    X = rng.uniform(-1, 1, (m, n))
    y = rng.uniform(-1, 1, n)
    run_hybrid_both("C1", X, y, lazy=(kind != "diag_rot"), kind=kind)


def test_ctmat_bit_exact():
    prm = O.Params.from_dict(W.params_dict("C1"))
    ctx = context("C1")
    N = prm.N
    sk_gpu = ctx.keygen(SEED_SK)
    s = O.keygen(prm, SEED_SK)
    rng = np.random.default_rng(8)
    A = rng.uniform(-1, 1, (16, 8))
    Wm = rng.normal(0, 0.1, (8, 5))
    plan = ctx.plan(3, 16, 8, n_out=5, pack=2)
    oplan = PL.CtMatPlan(16, 8, 5, prm.slots, 2)
    lv = prm.L
    Q = 2 * (lv + 1) * N
    ct = dev_f64(plan.bytes("ct_in") // 8)
    octs = []
    for i in range(oplan.ndiag):
        mi = O.encode(PL.ctmat_ct_slots(oplan, A, i), N, prm.scale)
        one = dev_f64(Q)
        ctx.encrypt_coeffs(sk_gpu, lv, dev_i64(mi), 100 + i, one)
        ct[i * Q:(i + 1) * Q] = one
        octs.append(O.encrypt(prm, s, mi, lv, 100 + i))
    pts = [O.encode(PL.ctmat_pt_slots(oplan, Wm, i, k), N, prm.scale)
           for i in range(oplan.ndiag) for k in range(oplan.n_out_cts)]
    pt = dev_f64(plan.bytes("pt") // 8)
    ctx.pt_import(lv, False, dev_i64(np.stack(pts)), pt)
    out = dev_f64(plan.bytes("ct_out") // 8)
    plan.matmul(ct, pt, None, out)
    got = export_ct(ctx, lv, out, oplan.n_out_cts)
    want = PL.ctmat_matmul(prm, oplan, octs, pts)
    for k, w in enumerate(want):
        assert_same(got[k, 0], w.c0, f"ctmat out {k} c0")
        assert_same(got[k, 1], w.c1, f"ctmat out {k} c1")


def test_row_plan_bit_exact():
    prm = O.Params.from_dict(W.params_dict("C2"))
    ctx = context("C2")
    N = prm.N
    sk_gpu = ctx.keygen(SEED_SK)
    s = O.keygen(prm, SEED_SK)
    rng = np.random.default_rng(9)
    m, n = 3, 8
    X = rng.standard_normal((m, n))
    y = rng.uniform(-1, 1, n)
    plan = ctx.plan(2, m, n)
    oplan = PL.RowPlan(m, n, prm.slots)
    lv = prm.L
    gal = plan.galois()
    assert sorted(gal) == PL.row_galois(oplan, N)
    keys = ctx.rotkeys(sk_gpu, gal, SEED_KEYS)
    okeys = {g: O.rotkey_gen(prm, s, g, SEED_KEYS) for g in gal}
    ct_slots = np.array([y[t % oplan.np_] if t % oplan.np_ < n else 0.0 for t in range(prm.slots)])
    mi = O.encode(ct_slots, N, prm.scale)
    ct = dev_f64(2 * (lv + 1) * N)
    ctx.encrypt_coeffs(sk_gpu, lv, dev_i64(mi), SEED_ENC, ct)
    oct_ = O.encrypt(prm, s, mi, lv, SEED_ENC)
    pts = [O.encode(PL.row_pt_slots(oplan, X, r), N, prm.scale) for r in range(m)]
    ind = np.zeros(prm.slots)
    ind[0] = 1.0
    ind_ints = O.encode(ind, N, float(prm.q[lv - 1]))
    pt = dev_f64(plan.bytes("pt") // 8)
    ctx.pt_import(lv, False, dev_i64(np.stack(pts + [ind_ints])), pt)
    out = dev_f64(plan.bytes("ct_out") // 8)
    plan.matmul(ct, pt, keys, out)
    got = export_ct(ctx, lv - 2, out)[0]
    want = PL.row_matmul(prm, oplan, oct_, pts, ind_ints, okeys)
    assert_same(got[0], want.c0, "row c0")
    assert_same(got[1], want.c1, "row c1")
    z = O.decrypt_decode(prm, s, want, prm.scale ** 2 / prm.q[lv])
    assert np.linalg.norm(z[:m] - X @ y) / np.linalg.norm(X @ y) < 2 ** -20


@pytest.mark.parametrize("name,m,n", [("C1", 16, 4), ("C1", 4, 16), ("C1", 8, 8), ("C4", 16, 4), ("C4", 4, 16)])
def test_transposed_conversion_bit_exact(name, m, n):
    """Eq. 7 (reading): the GPU's [[A^T]] diagonals equal the oracle's residue
    for residue (C4: three special primes, two digits)"""
    prm = O.Params.from_dict(W.params_dict(name))
    ctx = context(name)
    N, S, lv = prm.N, prm.slots, prm.L
    width = max(PL.pow2_ceil(m), PL.pow2_ceil(n))
    rng = np.random.default_rng(m * 3 + n)
    A = rng.uniform(-1, 1, (m, n))
    oplan = PL.CtMatPlan(m, n, 1, S, pack=S // width)
    plan = ctx.plan(pvfl.PLAN_CTMAT, m, n, n_out=1, pack=S // width)
    gal = plan.transpose_galois()
    assert gal == PL.transpose_galois(oplan, N)
    sk_gpu = ctx.keygen(SEED_SK)
    s = O.keygen(prm, SEED_SK)
    keys = ctx.rotkeys(sk_gpu, gal, SEED_KEYS) if gal else None
    okeys = {g: O.rotkey_gen(prm, s, g, SEED_KEYS) for g in gal}
    ct = dev_f64(plan.bytes("ct_in") // 8)
    octs = []
    Q2 = 2 * (lv + 1) * N
    for i in range(oplan.ndiag):
        mi = O.encode(PL.ctmat_ct_slots(oplan, A, i), N, prm.scale)
        one = dev_f64(Q2)
        ctx.encrypt_coeffs(sk_gpu, lv, dev_i64(mi), SEED_ENC + i, one)
        ct[i * Q2:(i + 1) * Q2] = one
        octs.append(O.encrypt(prm, s, mi, lv, SEED_ENC + i))
    out = dev_f64(plan.bytes("ct_in") // 8)
    plan.transpose(ct, keys, out)
    got = export_ct(ctx, lv, out, oplan.ndiag)
    want = PL.ctmat_transpose(prm, oplan, octs, okeys)
    for i, w in enumerate(want):
        assert_same(got[i, 0], w.c0, f"diag {i} c0")
        assert_same(got[i, 1], w.c1, f"diag {i} c1")


def test_transposed_conversion_rejects_partial_packing():
    ctx = context("C1")
    plan = ctx.plan(pvfl.PLAN_CTMAT, 16, 4, n_out=1, pack=1)
    with pytest.raises(pvfl.PvflError):
        plan.transpose_galois()


@pytest.mark.parametrize("m,n", [(16, 8), (100, 37), (4096, 3)])
def test_column_order_bit_exact(m, n):
    """Sec. 3.1's column-order method (n input ciphertexts, no rotation):
    residues equal the oracle's; counts are Table 2's column-order row"""
    prm = O.Params.from_dict(W.params_dict("C1"))
    ctx = context("C1")
    N, lv = prm.N, prm.L
    rng = np.random.default_rng(m * 11 + n)
    X = rng.uniform(-1, 1, (m, n))
    y = rng.uniform(-1, 1, n)
    plan = ctx.plan(4, m, n)
    oplan = PL.ColPlan(m, n, prm.slots)
    info = plan.info
    want_counts = oplan.op_counts()
    assert (info["n_mult"], info["n_add"], info["n_rot"], info["n_hstrot"], info["ct_in"], info["ct_out"]) == (
        want_counts["mult"], want_counts["add"], 0, 0, n, oplan.row_blocks)
    sk = ctx.keygen(SEED_SK)
    s = O.keygen(prm, SEED_SK)
    ct = dev_f64(plan.bytes("ct_in") // 8)
    octs = []
    for j in range(n):
        mi = O.encode(PL.col_ct_slots(oplan, y, j), N, prm.scale)
        one = dev_f64(2 * (lv + 1) * N)
        ctx.encrypt_coeffs(sk, lv, dev_i64(mi), SEED_ENC + j, one)
        ct[j * 2 * (lv + 1) * N:(j + 1) * 2 * (lv + 1) * N] = one
        octs.append(O.encrypt(prm, s, mi, lv, SEED_ENC + j))
    pts = PL.col_pt_ints(prm, oplan, X, prm.scale)
    pt = dev_f64(plan.bytes("pt") // 8)
    ctx.pt_import(lv, False, dev_i64(np.stack(pts)), pt)
    out = dev_f64(plan.bytes("ct_out") // 8)
    plan.matmul(ct, pt, None, out)
    got = export_ct(ctx, lv, out, info["ct_out"])
    want = PL.col_matmul(prm, oplan, octs, pts)
    for b, w in enumerate(want):
        assert_same(got[b, 0], w.c0, f"out {b} c0")
        assert_same(got[b, 1], w.c1, f"out {b} c1")


def test_column_order_real_path():
    """encode, encrypt (one ciphertext per column), product, decrypt and read
    out on the GPU: within 2^-20 of X y"""
    import torch
    ctx = context("C1")
    XT, r = W.c1_inputs()
    m, n = XT.shape
    f64 = dict(dtype=torch.float64, device="cuda")
    plan = ctx.plan(4, m, n)
    sk = ctx.keygen(SEED_SK)
    pt = torch.empty(plan.bytes("pt") // 8, **f64)
    plan.encode_pt(torch.from_numpy(XT).to(**f64), pt)
    ct = torch.empty(plan.bytes("ct_in") // 8, **f64)
    plan.encrypt(sk, torch.from_numpy(r).to(**f64), SEED_ENC, ct)
    out = torch.empty(plan.bytes("ct_out") // 8, **f64)
    plan.matmul(ct, pt, None, out)
    y = torch.empty(m, **f64)
    plan.decrypt_decode(sk, out, y)
    ref = XT @ r
    assert np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref) < 2.0 ** -20
