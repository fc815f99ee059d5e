"""The real-valued path on the GPU: encode -> encrypt -> matmul -> decrypt,
decode, lazy RaS.  Encoders use independent FP64 FFTs, so rounded
coefficients may differ by one where the exact value sits next to a .5
boundary; everything from the integer plaintext on is compared bit for bit
elsewhere.  Needs an MI355X."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import plans as PL
from paper_2405_00482_amd import pvfl
from paper_2405_00482_amd import workloads as W

from gpu_util import context, dev_f64, export, export_ct, torch

pytestmark = pytest.mark.gpu


def to_dev(a):
    return torch().from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def signed_diff(a, b, q):
    d = (a.astype(object) - b.astype(object)) % q
    return np.array([int(x) if x <= q // 2 else int(x) - q for x in d.ravel()], dtype=np.int64).reshape(a.shape)


@pytest.mark.parametrize("name,m,n,bs", [("C1", 16, 256, 0), ("C2", 256, 1024, 0), ("C1", 100, 37, 0),
                                         ("C2", 256, 1024, 8), ("C5", 40, 1000, 0)])
def test_encode_pt_within_one_of_oracle(name, m, n, bs):
    prm = O.Params.from_dict(W.params_dict(name))
    ctx = context(name)
    rng = np.random.default_rng(m)
    X = rng.standard_normal((m, n))
    plan = ctx.plan(0, m, n, lazy=True, bsgs=bs)
    oplan = PL.HybridPlan(m, n, prm.slots)
    pt = dev_f64(plan.bytes("pt") // 8)
    plan.encode_pt(to_dev(X), pt)
    K = plan.info["pt_limbs"]
    got = export(ctx, prm.L, True, pt, plan.info["n_pts"])
    want = PL.bsgs_pt_ints(prm, oplan, X, prm.scale, bs) if bs else PL.hybrid_pt_ints(prm, oplan, X, prm.scale)
    n_diff = 0
    for k, mk in enumerate(want):
        for l, q in enumerate(prm.qp(prm.L)):
            d = signed_diff(got[k, l], O.poly_from_signed(mk, q), q)
            assert np.abs(d).max() <= 1, (k, l)
            if l == 0:
                n_diff += int(np.count_nonzero(d))
        # every limb must carry the same integer vector
        d0 = signed_diff(got[k, 0], O.poly_from_signed(mk, prm.q[0]), prm.q[0])
        for l, q in enumerate(prm.qp(prm.L)):
            assert np.array_equal(signed_diff(got[k, l], O.poly_from_signed(mk, q), q), d0)
    frac = n_diff / (len(want) * prm.N)
    assert frac < 0.05, frac
    print(f"encode {name} {m}x{n}: {n_diff} of {len(want) * prm.N} coefficients differ by one ({frac:.2e})")


def test_encrypt_real_matches_oracle():
    prm = O.Params.from_dict(W.params_dict("C1"))
    ctx = context("C1")
    XT, r = W.c1_inputs()
    plan = ctx.plan(0, 16, 256, lazy=True)
    oplan = PL.HybridPlan(16, 256, prm.slots)
    sk = ctx.keygen(3)
    s = O.keygen(prm, 3)
    ct = dev_f64(plan.bytes("ct_in") // 8)
    plan.encrypt(sk, to_dev(r), 77, ct)
    got = export_ct(ctx, prm.L, ct)[0]
    mi = PL.hybrid_ct_ints(prm, oplan, r, prm.scale)[0]
    want = O.encrypt(prm, s, mi, prm.L, 77)
    assert np.array_equal(got[1], want.c1)
    for l, q in enumerate(prm.q):
        assert np.abs(signed_diff(got[0, l], want.c0[l], q)).max() <= 1


@pytest.mark.parametrize("name,lazy,bs", [("C1", True, 0), ("C1", False, 0), ("C2", True, 0), ("C2", True, 8)])
def test_hybrid_real_path_precision(name, lazy, bs):
    prm = O.Params.from_dict(W.params_dict(name))
    ctx = context(name)
    XT, r = W.c1_inputs() if name == "C1" else W.c2_inputs()
    m, n = XT.shape
    plan = ctx.plan(0, m, n, lazy=lazy, bsgs=bs)
    sk = ctx.keygen(5)
    keys = ctx.rotkeys(sk, plan.galois(), 6)
    pt = dev_f64(plan.bytes("pt") // 8)
    ct = dev_f64(plan.bytes("ct_in") // 8)
    out = dev_f64(plan.bytes("ct_out") // 8)
    y = dev_f64(m)
    plan.encode_pt(to_dev(XT), pt)
    plan.encrypt(sk, to_dev(r), 9, ct)
    plan.matmul(ct, pt, keys, out)
    plan.decrypt_decode(sk, out, y)
    got = y.cpu().numpy()
    ref = XT @ r
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"{name} lazy={lazy} bsgs={bs}: rel err 2^{np.log2(err):.2f}")
    assert err < (2.0 ** -20 if lazy else 2.0 ** -18)


def test_decode_matches_oracle_decoder():
    """GPU decrypt+decode of an exactly known ciphertext equals the oracle's
    decoding of the same residues to FP64 rounding."""
    prm = O.Params.from_dict(W.params_dict("C1"))
    ctx = context("C1")
    plan = ctx.plan(1, 64, 64, lazy=True)   # DIAG, m = n: slot j holds row j
    sk = ctx.keygen(4)
    s = O.keygen(prm, 4)
    rng = np.random.default_rng(5)
    z = rng.uniform(-1, 1, prm.slots)
    scale2 = 2.0 ** plan.info["out_log2_scale"]
    mi = O.encode(z, prm.N, scale2 / 2 ** 25)   # keep |m| well inside int64
    ct = dev_f64(2 * (prm.L + 1) * prm.N)
    from gpu_util import dev_i64
    ctx.encrypt_coeffs(sk, prm.L, dev_i64(mi), 8, ct)
    y = dev_f64(64)
    plan.decrypt_decode(sk, ct, y)
    want = O.decrypt_decode(prm, s, O.encrypt(prm, s, mi, prm.L, 8), scale2)[:64]
    np.testing.assert_allclose(y.cpu().numpy(), want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind,m,n", [("diag", 64, 16), ("diag", 16, 64), ("diag_rot", 16, 64), ("row", 6, 16)])
def test_other_plans_real_path(kind, m, n):
    name = "C2" if kind == "row" else "C1"
    ctx = context(name)
    rng = np.random.default_rng(11)
    X = rng.uniform(-1, 1, (m, n))
    yv = rng.uniform(-1, 1, n)
    k = {"diag": 1, "diag_rot": 1, "row": 2}[kind]
    plan = ctx.plan(k, m, n, lazy=(kind == "diag"), ras_in_ct=(kind == "diag_rot"))
    sk = ctx.keygen(1)
    keys = ctx.rotkeys(sk, plan.galois(), 2)
    pt = dev_f64(plan.bytes("pt") // 8)
    ct = dev_f64(plan.bytes("ct_in") // 8)
    out = dev_f64(plan.bytes("ct_out") // 8)
    y = dev_f64(m)
    plan.encode_pt(to_dev(X), pt)
    plan.encrypt(sk, to_dev(yv), 3, ct)
    plan.matmul(ct, pt, keys, out)
    plan.decrypt_decode(sk, out, y)
    ref = X @ yv
    err = np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err < 2.0 ** -18, err


@pytest.mark.parametrize("pack", [1, 32])
def test_ctmat_real_path(pack):
    """C4 shapes: [[H]] (256 x 64) W (64 x 256) and [[delta]] (256 x 256) W^T."""
    ctx = context("C4")
    H, Wm, delta = W.c4_inputs()
    for A, B in ((H, Wm), (delta, np.ascontiguousarray(Wm.T))):
        m, n = A.shape
        nout = B.shape[1]
        p = min(pack, (ctx.N // 2) // max(m, n))
        plan = ctx.plan(3, m, n, n_out=nout, pack=p)
        sk = ctx.keygen(1)
        pt = dev_f64(plan.bytes("pt") // 8)
        ct = dev_f64(plan.bytes("ct_in") // 8)
        out = dev_f64(plan.bytes("ct_out") // 8)
        y = dev_f64(m * nout)
        plan.encode_pt(to_dev(B), pt)
        plan.encrypt(sk, to_dev(A), 3, ct)
        plan.matmul(ct, pt, None, out)
        plan.decrypt_decode(sk, out, y)
        ref = A @ B
        err = np.linalg.norm(y.cpu().numpy().reshape(m, nout) - ref) / np.linalg.norm(ref)
        assert err < 2.0 ** -20, err


def test_ring_2_15_full_size_product():
    """The large workload at full size: X^T (5000 x 4096, 90% zeros) times one
    encrypted column of R at N = 2^15 with 8+2 primes -- m' = 2048, 2047
    hoisted rotations over a 40 GiB key set.  The decrypted product must be
    within 2^-20 of the FP64 product (every output, norm-wise)."""
    t = torch()
    name = "C5"
    ctx = context(name)
    XT, R = W.c5_inputs(cols=[0])
    r = np.ascontiguousarray(R[:, 0])
    m, n = XT.shape
    plan = ctx.plan(0, m, n, lazy=True)
    assert plan.info["mprime"] == 2048 and plan.info["n_galois"] == 2047
    seeds = W.seeds(name)
    sk = ctx.keygen(seeds["sk"])
    keys = ctx.rotkeys(sk, plan.galois(), seeds["rotkeys"])
    pt = dev_f64(plan.bytes("pt") // 8)
    ct = dev_f64(plan.bytes("ct_in") // 8)
    out = dev_f64(plan.bytes("ct_out") // 8)
    y = dev_f64(m)
    plan.encode_pt(to_dev(XT), pt)
    plan.encrypt(sk, to_dev(r), seeds["enc"], ct)
    plan.matmul(ct, pt, keys, out)
    plan.decrypt_decode(sk, out, y)
    got = y.cpu().numpy()
    ref = XT @ r
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"C5 full size: rel err 2^{np.log2(err):.2f}")
    assert err < 2.0 ** -20
    del keys
    t.cuda.empty_cache()


def test_vfl_nn_backward_via_transposed_conversion():
    """VFL-NN layer at C4 (Sec. 5.3): [[H]] (256 x 64) sent once as Eq. 5
    diagonals; forward [[H]] W by Alg. 3, backward H^T delta^T by converting
    [[H]] to [[H^T]] (Eq. 7) and Alg. 3 again.  Both within 2^-20."""
    ctx = context("C4")
    H, Wm, _ = W.c4_inputs()
    rng = np.random.default_rng(44)
    D = rng.uniform(-1, 1, (H.shape[0], 32))          # delta_act^T: batch x n'
    m, n = H.shape
    width = max(m, n)
    pack = (ctx.N // 2) // width
    fwd = ctx.plan(pvfl.PLAN_CTMAT, m, n, n_out=Wm.shape[1], pack=pack)
    bwd = ctx.plan(pvfl.PLAN_CTMAT, n, m, n_out=D.shape[1], pack=pack)
    sk = ctx.keygen(9)
    keys = ctx.rotkeys(sk, fwd.transpose_galois(), 10)
    ct = dev_f64(fwd.bytes("ct_in") // 8)
    fwd.encrypt(sk, to_dev(H), 11, ct)
    for plan, B, ct_in, ref in ((fwd, Wm, ct, H @ Wm), (bwd, D, None, H.T @ D)):
        if ct_in is None:
            ct_in = dev_f64(bwd.bytes("ct_in") // 8)
            fwd.transpose(ct, keys, ct_in)
        pt = dev_f64(plan.bytes("pt") // 8)
        out = dev_f64(plan.bytes("ct_out") // 8)
        y = dev_f64(ref.size)
        plan.encode_pt(to_dev(B), pt)
        plan.matmul(ct_in, pt, None, out)
        plan.decrypt_decode(sk, out, y)
        got = y.cpu().numpy().reshape(ref.shape)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"{'forward' if plan is fwd else 'backward'}: rel err 2^{np.log2(err):.2f}")
        assert err < 2.0 ** -20


@pytest.mark.parametrize("kind,lazy,o3", [("diag", True, False), ("diag", False, False), ("diag", False, True),
                                          ("hybrid", False, True), ("row", False, False)])
def test_c2_full_size_other_plans(kind, lazy, o3):
    """The logistic-regression gradient at its full size (X^T 256 x 1024 times
    [[r]], N = 2^13, 3+1 primes) by the diagonal (Eq. 5), GALA-style (O3) and
    row-wise (Sec. 3.1, 2815 rotations and two rescales) plans: every output
    within 2^-20 of the FP64 product"""
    ctx = context("C2")
    XT, r = W.c2_inputs()
    m, n = XT.shape
    k = {"hybrid": 0, "diag": 1, "row": 2}[kind]
    plan = ctx.plan(k, m, n, lazy=lazy, unhoisted=o3)
    if kind == "row":
        assert plan.info["n_rot"] == m * 10 + m - 1
    sk = ctx.keygen(5)
    keys = ctx.rotkeys(sk, plan.galois(), 6)
    pt = dev_f64(plan.bytes("pt") // 8)
    ct = dev_f64(plan.bytes("ct_in") // 8)
    out = dev_f64(plan.bytes("ct_out") // 8)
    y = dev_f64(m)
    plan.encode_pt(to_dev(XT), pt)
    plan.encrypt(sk, to_dev(r), 9, ct)
    plan.matmul(ct, pt, keys, out)
    plan.decrypt_decode(sk, out, y)
    ref = XT @ r
    err = np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"C2 {kind} lazy={lazy} o3={o3}: rel err 2^{np.log2(err):.2f}")
    assert err < 2.0 ** -20
