"""Sec. 5.2 on the GPU, through the C ABI: the summed product of Eq. 4, the
cleartext at the output scale (inverse RaS and slot masks), the plaintext
addition and the masking party's rotate-and-sum; against the oracle.  Needs an
MI355X."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import plans as PL
from paper_2405_00482_amd import pvfl
from paper_2405_00482_amd import workloads as W

from gpu_util import context, dev_f64, dev_i64, export, export_ct, first_mismatch

pytestmark = pytest.mark.gpu

SEED_SK, SEED_KEYS = 41, 42


def assert_same(got, want, what):
    mm = first_mismatch(np.asarray(got, dtype=np.uint64), np.asarray(want, dtype=np.uint64))
    assert mm is None, f"{what}: first mismatch at {mm[0]} gpu={mm[1]} oracle={mm[2]} ({mm[3]} differ)"


def _terms(prm, oplan, kind, Xs, ys):
    N = prm.N
    out = []
    for X, y in zip(Xs, ys):
        if kind == "hybrid":
            out.append((PL.hybrid_pt_ints(prm, oplan, X, prm.scale), PL.hybrid_ct_ints(prm, oplan, y, prm.scale)))
        else:
            out.append(([O.encode(PL.diag_pt_slots(oplan, X, i), N, prm.scale) for i in range(oplan.ndiag)],
                        [O.encode(PL.diag_ct_slots(oplan, y), N, prm.scale)]))
    return out


@pytest.mark.parametrize("kind,m,n", [("hybrid", 16, 256), ("hybrid", 4, 4096), ("hybrid", 4096, 4),
                                      ("hybrid", 1, 1), ("diag", 16, 64)])
def test_matmul_sum_bit_exact(kind, m, n):
    """two terms of one layout summed over Q u P, one ModDown per output (Eq. 4)"""
    prm = O.Params.from_dict(W.params_dict("C1"))
    ctx = context("C1")
    N, lv = prm.N, prm.L
    rng = np.random.default_rng(m * 5 + n)
    Xs = [rng.uniform(-1, 1, (m, n)) for _ in range(2)]
    ys = [rng.uniform(-1, 1, n) for _ in range(2)]
    plan = ctx.plan(0 if kind == "hybrid" else 1, m, n, lazy=True)
    oplan = PL.HybridPlan(m, n, prm.slots) if kind == "hybrid" else PL.DiagPlan(m, n, prm.slots)
    sk = ctx.keygen(SEED_SK)
    s = O.keygen(prm, SEED_SK)
    gal = plan.galois()
    keys = ctx.rotkeys(sk, gal, SEED_KEYS) if gal else None
    okeys = {g: O.rotkey_gen(prm, s, g, SEED_KEYS) for g in gal}
    info = plan.info
    cts, pts, oterms = [], [], []
    for t, (pt_ints, ct_ints) in enumerate(_terms(prm, oplan, kind, Xs, ys)):
        ct = dev_f64(plan.bytes("ct_in") // 8)
        octs = []
        for c, mi in enumerate(ct_ints):
            one = dev_f64(2 * (lv + 1) * N)
            seed = 100 * t + c
            ctx.encrypt_coeffs(sk, lv, dev_i64(mi), seed, one)
            ct[c * 2 * (lv + 1) * N:(c + 1) * 2 * (lv + 1) * N] = one
            octs.append(O.encrypt(prm, s, mi, lv, seed))
        pt = dev_f64(plan.bytes("pt") // 8)
        ctx.pt_import(lv, info["pt_limbs"] > lv + 1, dev_i64(np.stack(pt_ints)), pt)
        cts.append(ct)
        pts.append(pt)
        oterms.append((octs, pt_ints))
    out = dev_f64(plan.bytes("ct_out") // 8)
    ws = dev_f64(plan.workspace_sum_bytes(2) // 8)
    plan.matmul_sum(cts, pts, keys, out, ws)
    got = export_ct(ctx, lv, out, info["ct_out"])
    want = PL.hybrid_matmul_sum(prm, oplan, oterms, okeys)
    for b, w in enumerate(want):
        assert_same(got[b, 0], w.c0, f"out {b} c0")
        assert_same(got[b, 1], w.c1, f"out {b} c1")


def test_matmul_sum_rejects_other_plans():
    ctx = context("C1")
    for p in (ctx.plan(0, 16, 256, lazy=False), ctx.plan(0, 64, 256, lazy=True, bsgs=2),
              ctx.plan(1, 16, 64, lazy=True, ras_in_ct=True), ctx.plan(3, 16, 64, n_out=4)):
        t = dev_f64(max(p.bytes("ct_in"), p.bytes("pt"), p.bytes("ct_out")) // 8)
        with pytest.raises(pvfl.PvflError):
            p.matmul_sum([t], [t], None, t)


def _inv_mod(a, q):
    return pow(int(a), -1, int(q))


@pytest.mark.parametrize("kind,m,n,mode", [("hybrid", 16, 256, 0), ("hybrid", 4096, 4, 0), ("diag", 16, 64, 0),
                                           ("ctmat", 16, 64, 0), ("hybrid", 16, 256, 1)])
def test_encode_out_matches_oracle(kind, m, n, mode):
    """the output-scale plaintext: its residues divided by 2^e equal the oracle's
    integer coefficients (of the oracle's inverse-RaS slots) within one -- two
    independent FP64 encoders may round a coefficient differently"""
    prm = O.Params.from_dict(W.params_dict("C1"))
    ctx = context("C1")
    N = prm.N
    rng = np.random.default_rng(m + 7 * n + mode)
    if kind == "ctmat":
        plan = ctx.plan(3, m, n, n_out=3, pack=2)
        oplan = PL.CtMatPlan(m, n, 3, prm.slots, pack=2)
        v = rng.uniform(-4, 4, m * 3)
    else:
        plan = ctx.plan(0 if kind == "hybrid" else 1, m, n, lazy=True)
        oplan = PL.HybridPlan(m, n, prm.slots) if kind == "hybrid" else PL.DiagPlan(m, n, prm.slots)
        v = rng.uniform(-4, 4, m)
    info = plan.info
    lv = info["out_level"]
    e = int(round(info["out_log2_scale"] - prm.log2_scale))
    if mode == 1:
        v = rng.uniform(-8, 8, info["ct_out"] * prm.slots)
        slots = [v[b * prm.slots:(b + 1) * prm.slots] for b in range(info["ct_out"])]
    else:
        slots = PL.out_slots(oplan, v)
    pt = dev_f64(plan.bytes("pt_out") // 8)
    vd = dev_f64(v.size)
    vd.copy_(vd.new_tensor(v))
    plan.encode_out(vd, mode, pt)
    got = export(ctx, lv, False, pt, info["ct_out"])
    for b, z in enumerate(slots):
        want = O.encode(z, N, prm.scale)
        for i, q in enumerate(prm.q[: lv + 1]):
            r = (got[b, i].astype(object) * _inv_mod(pow(2, e, q), q)) % q
            r = np.where(r > q // 2, r - q, r).astype(np.int64)
            d = np.abs(r - want)
            assert d.max() <= 1, f"limb {i}: {int(d.max())}"
            assert (d > 0).mean() < 0.01


def test_out_add_pt_and_lazy_ras():
    """ct +- pt is exact residue arithmetic on c0 (c1 unchanged): residues
    equal the oracle's ct_add_plain on the oracle's ciphertext and the same
    integer plaintext; the masking party's RaS equals the oracle's"""
    prm = O.Params.from_dict(W.params_dict("C1"))
    ctx = context("C1")
    N, lv = prm.N, prm.L
    plan = ctx.plan(0, 16, 256, lazy=True)
    oplan = PL.HybridPlan(16, 256, prm.slots)
    sk = ctx.keygen(SEED_SK)
    s = O.keygen(prm, SEED_SK)
    rng = np.random.default_rng(5)
    m_ints = rng.integers(-2 ** 40, 2 ** 40, N)
    ct = dev_f64(plan.bytes("ct_out") // 8)
    ctx.encrypt_coeffs(sk, lv, dev_i64(m_ints), 7, ct)
    oct_ = O.encrypt(prm, s, m_ints, lv, 7)
    p_ints = rng.integers(-2 ** 45, 2 ** 45, N)
    pt = dev_f64(plan.bytes("pt_out") // 8)
    ctx.pt_import(lv, False, dev_i64(p_ints[None, :]), pt)
    p_res = O.reduce_signed(p_ints, prm.q[: lv + 1])
    for sign in (1, -1):
        out = dev_f64(plan.bytes("ct_out") // 8)
        plan.out_add_pt(ct, pt, sign, out)
        o = export_ct(ctx, lv, out)[0]
        want = PL.ct_add_plain(prm, oct_, p_res, sign)
        assert_same(o[0], want.c0, f"c0 sign {sign}")
        assert_same(o[1], want.c1, f"c1 sign {sign}")
    mask = rng.uniform(-8, 8, prm.slots)
    mask_dev = dev_f64(prm.slots)
    mask_dev.copy_(mask_dev.new_tensor(mask))
    y = dev_f64(16)
    plan.lazy_ras(mask_dev, y)
    np.testing.assert_allclose(y.cpu().numpy(), PL.hybrid_lazy_ras(oplan, [mask]), rtol=0, atol=1e-12)


@pytest.mark.parametrize("name,batch,features", [("C3", 1024, 64), ("C2", 300, 40)])
def test_caesar_gradient_eq4_masked(name, batch, features):
    """CAESAR's [[g_B]] by Eq. 4 on the whole GPU path: [[z]] and [[z^3]] times
    the plaintexts q1 X^T and q2 X^T in one summed product (one level), the
    cleartext (q0 1 - y)^T X added through the inverse RaS, a random slot mask
    subtracted; the two shares add up to the cleartext gradient within 2^-20."""
    import torch
    prm = O.Params.from_dict(W.params_dict(name))
    ctx = context(name)
    rng = np.random.default_rng(batch + features)
    XB = rng.standard_normal((batch, features))
    XB = (XB - XB.mean(axis=0)) / XB.std(axis=0)
    z = rng.uniform(-2, 2, batch)
    y = rng.integers(0, 2, batch).astype(float)
    q0, q1, q2 = 0.5, 0.197, -0.004           # the degree-3 sigmoid approximation CAESAR uses
    want, _ = PL.eq4_cleartext(q0, q1, q2, z, y, XB)
    f64 = dict(dtype=torch.float64, device="cuda")
    XT = torch.from_numpy(np.ascontiguousarray(XB.T)).to(**f64)
    plan = ctx.plan(0, features, batch, lazy=True)
    sk = ctx.keygen(SEED_SK)
    keys = ctx.rotkeys(sk, plan.galois(), SEED_KEYS) if plan.galois() else None
    cts, pts = [], []
    for k, (coef, vec) in enumerate(((q1, z), (q2, z ** 3))):
        pt = torch.empty(plan.bytes("pt") // 8, **f64)
        plan.encode_pt(XT, pt, coef=coef)
        ct = torch.empty(plan.bytes("ct_in") // 8, **f64)
        plan.encrypt(sk, torch.from_numpy(vec).to(**f64), 900 + k, ct)
        cts.append(ct)
        pts.append(pt)
    out = torch.empty(plan.bytes("ct_out") // 8, **f64)
    plan.matmul_sum(cts, pts, keys, out)
    clear = torch.from_numpy((q0 * np.ones(batch) - y) @ XB).to(**f64)
    ptc = torch.empty(plan.bytes("pt_out") // 8, **f64)
    plan.encode_out(clear, pvfl.OUT_ROWS, ptc)
    plan.out_add_pt(out, ptc, 1, out)
    mask = torch.from_numpy(rng.uniform(-8, 8, plan.info["ct_out"] * prm.slots)).to(**f64)
    ptm = torch.empty(plan.bytes("pt_out") // 8, **f64)
    plan.encode_out(mask, pvfl.OUT_SLOTS, ptm)
    plan.out_add_pt(out, ptm, -1, out)
    share_b = torch.empty(features, **f64)
    plan.decrypt_decode(sk, out, share_b)
    share_a = torch.empty(features, **f64)
    plan.lazy_ras(mask, share_a)
    got = (share_a + share_b).cpu().numpy()
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err < 2.0 ** -20, err
    # the masked share alone is far from the gradient
    assert np.linalg.norm(share_b.cpu().numpy() - want) / np.linalg.norm(want) > 1e-2
