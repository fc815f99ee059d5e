"""Pins of the CPU oracle against facts fixed outside it: published known-answer
vectors, closed forms, brute force at tiny sizes, exact big-integer identities
and the paper's worked examples.  CPU only."""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from oracle import plans as PL
from paper_2405_00482_amd import workloads as W

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

Q40 = 1099511480321      # 1 mod 2^13, prime, below 2^40
Q48 = 281474976694273    # 1 mod 2^13, prime, below 2^48


def tiny_params(logN=4, nq=3, npr=1, alpha=None):
    """Small ring with real NTT-friendly primes."""
    N = 1 << logN
    qs = []
    x = ((1 << 40) - 1) // (2 * N) * (2 * N) + 1
    while len(qs) < nq + npr:
        if O.is_prime(x):
            qs.append(x)
        x -= 2 * N
    return O.Params(logN=logN, q=qs[:nq], p=qs[nq:], log2_scale=20.0)


# --------------------------------------------------------------------------
# PRNG
# --------------------------------------------------------------------------
def test_philox_known_answers():
    d = json.load(open(os.path.join(GOLD, "philox_kat.json")))
    for v in d["vectors"]:
        out = O.philox4x32_10([int(x, 16) for x in v["ctr"]], [int(x, 16) for x in v["key"]])
        assert ["%08x" % x for x in out] == v["out"]


def test_sampler_ranges_and_moments():
    N = 1 << 14
    u = O.sample_uniform(5, O.stream_enc_a(0), Q40, N)
    assert int(u.max()) < Q40
    assert abs(float(u.astype(np.float64).mean()) / Q40 - 0.5) < 0.02
    t = O.sample_ternary(5, O.stream_secret(), N)
    assert set(np.unique(t).tolist()) == {-1, 0, 1}
    assert abs(np.mean(t == 0) - 1 / 3) < 0.02
    e = O.sample_cbd21(5, O.stream_enc_e(), N)
    assert np.abs(e).max() <= 21
    assert abs(np.var(e) - 10.5) < 0.6          # CBD(eta) variance = eta / 2
    # word pairing of the generator: index 2k and 2k+1 come from one Philox block
    w = O.philox4x32_10([3, 0, 7, 0], [9, 0])
    assert O.rand64(9, 7, 6) == w[0] | (w[1] << 32)
    assert O.rand64(9, 7, 7) == w[2] | (w[3] << 32)


def test_sampler_mappings_from_raw_words():
    """Each sample is fixed by its raw 64-bit word u = rand64(seed, stream, i),
    itself pinned by the published Philox vectors above.  Uniform mod q is the
    top of the 128-bit product u q: x 2^64 <= u q < (x + 1) 2^64, so samples
    grow with u (a remainder u mod q would not); ternary splits [0, 2^64)
    into thirds; CBD(21) is the difference of the bit counts of u's two low
    21-bit fields.  Checked with exact Python integers on every index."""
    n = 4096
    seed, st = 77, O.stream_enc_a(3)
    words = [O.rand64(seed, st, i) for i in range(n)]
    for q in (Q40, Q48, 3):
        x = O.sample_uniform(seed, st, q, n)
        for u, v in zip(words, x.tolist()):
            assert v * 2 ** 64 <= u * q < (v + 1) * 2 ** 64
        order = np.argsort(np.array(words, dtype=np.uint64), kind="stable")
        assert np.all(np.diff(x[order].astype(np.int64)) >= 0), "uniform samples must grow with the raw word"
    t = O.sample_ternary(seed, st, n)
    for u, v in zip(words, t.tolist()):
        assert (v + 1) * 2 ** 64 <= 3 * u < (v + 2) * 2 ** 64
    e = O.sample_cbd21(seed, st, n)
    for u, v in zip(words, e.tolist()):
        lo, hi = u & (2 ** 21 - 1), (u >> 21) & (2 ** 21 - 1)
        assert v == bin(lo).count("1") - bin(hi).count("1")


# --------------------------------------------------------------------------
# NTT and negacyclic products
# --------------------------------------------------------------------------
@pytest.mark.parametrize("q", [Q40, Q48])
def test_psi_is_primitive_2n_root(q):
    for N in (16, 4096):
        psi = O.psi(q, N)
        assert pow(psi, N, q) == q - 1
        assert pow(psi, 2 * N, q) == 1


@pytest.mark.parametrize("N", [8, 64, 1024])
def test_ntt_roundtrip_and_closed_form(N):
    q = Q40
    rng = np.random.default_rng(N)
    a = rng.integers(0, q, size=N, dtype=np.uint64)
    assert np.array_equal(O.ntt_inverse(O.ntt_forward(a, q), q), a)
    psi = O.psi(q, N)
    for t in (0, 1, N - 1, N // 3):
        mono = np.zeros(N, dtype=np.uint64)
        mono[t] = 1
        A = O.ntt_forward(mono, q)
        for k in (0, 1, N // 2, N - 1):
            assert int(A[k]) == pow(psi, (2 * k + 1) * t, q)


@pytest.mark.parametrize("N", [4, 16, 64])
def test_ntt_product_matches_schoolbook(N):
    for q in (Q40, Q48):
        rng = np.random.default_rng(q % 1000 + N)
        a = rng.integers(0, q, size=N, dtype=np.uint64)
        b = rng.integers(0, q, size=N, dtype=np.uint64)
        assert np.array_equal(O.poly_mul(a, b, q), O.poly_mul_schoolbook(a, b, q))


def test_ntt_product_sparse_full_size():
    # random sparse operands at N = 2^14 against a Python-integer negacyclic sum
    N, q = 1 << 14, 281474976546817   # 1 mod 2^15
    rng = np.random.default_rng(3)
    a = np.zeros(N, dtype=np.uint64)
    b = np.zeros(N, dtype=np.uint64)
    ia = rng.choice(N, 6, replace=False)
    ib = rng.choice(N, 5, replace=False)
    a[ia] = rng.integers(0, q, 6, dtype=np.uint64)
    b[ib] = rng.integers(0, q, 5, dtype=np.uint64)
    want = [0] * N
    for i in ia:
        for j in ib:
            k = int(i) + int(j)
            v = int(a[i]) * int(b[j])
            if k < N:
                want[k] += v
            else:
                want[k - N] -= v
    assert [x % q for x in want] == [int(x) for x in O.poly_mul(a, b, q)]


def test_cheetah_coefficient_example():
    """Sec. 3.2: X~[i n + n - 1 - j] = X[i, j], y~[i] = y[i] in Z_q[X]/(X^16+1);
    coefficient i n + n - 1 of the product is row i of X dotted with y."""
    d = json.load(open(os.path.join(GOLD, "paper_examples.json")))["cheetah"]
    N, m, n = d["N"], d["m"], d["n"]
    q = Q40
    rng = np.random.default_rng(11)
    X = rng.integers(0, 1000, size=(m, n))
    y = rng.integers(0, 1000, size=n)
    xt = np.zeros(N, dtype=np.uint64)
    yt = np.zeros(N, dtype=np.uint64)
    for i in range(m):
        for j in range(n):
            xt[i * n + n - 1 - j] = X[i, j]
    yt[:n] = y
    prod = O.poly_mul(xt, yt, q)
    for i in range(m):
        assert int(prod[i * n + n - 1]) == int(X[i] @ y)


# --------------------------------------------------------------------------
# automorphisms
# --------------------------------------------------------------------------
def test_automorphism_monomials_and_composition():
    N, q = 64, Q40
    for g in (5, 25, 2 * N - 1, 3):
        for j in range(N):
            mono = np.zeros(N, dtype=np.uint64)
            mono[j] = 7
            out = O.automorphism(mono, g, q)
            e = (j * g) % (2 * N)
            want = np.zeros(N, dtype=np.uint64)
            if e < N:
                want[e] = 7
            else:
                want[e - N] = q - 7
            assert np.array_equal(out, want)
    rng = np.random.default_rng(5)
    a = rng.integers(0, q, size=N, dtype=np.uint64)
    b = rng.integers(0, q, size=N, dtype=np.uint64)
    g, h = 5, 125
    assert np.array_equal(O.automorphism(O.automorphism(a, g, q), h, q), O.automorphism(a, g * h % (2 * N), q))
    # ring homomorphism, product by schoolbook
    assert np.array_equal(O.automorphism(O.poly_mul_schoolbook(a, b, q), g, q),
                          O.poly_mul_schoolbook(O.automorphism(a, g, q), O.automorphism(b, g, q), q))


def test_five_has_order_n_over_two():
    for N in (16, 4096, 1 << 15):
        x, k = 5, 1
        while x != 1:
            x = x * 5 % (2 * N)
            k += 1
        assert k == N // 2
        assert O.galois_rotl(N // 2, N) == 1
        assert O.galois_rotl(3, N) * O.galois_rotr(3, N) % (2 * N) == 1


# --------------------------------------------------------------------------
# base conversion, ModDown, rescale (exact big-integer identities)
# --------------------------------------------------------------------------
def _crt(vals, primes):
    Q = math.prod(primes)
    x = 0
    for v, q in zip(vals, primes):
        Qi = Q // q
        x += int(v) * Qi * pow(Qi % q, -1, q)
    return x % Q


def test_base_conversion_overshoot_bound():
    prm = tiny_params(4, 3, 2)
    B = prm.q
    r = prm.p[0]
    rng = np.random.default_rng(7)
    N = prm.N
    limbs = [rng.integers(0, b, size=N, dtype=np.uint64) for b in B]
    conv = O.base_convert(limbs, B, r)
    Bint = math.prod(B)
    for k in range(N):
        X = _crt([l[k] for l in limbs], B)
        ok = [u for u in range(len(B)) if (int(conv[k]) - X - u * Bint) % r == 0]
        assert ok, "Conv(x) must equal x + u*B for some 0 <= u < |B|"


def test_moddown_is_rounded_division():
    prm = tiny_params(4, 3, 2)          # alpha = 2
    lv = prm.L
    basis = prm.qp(lv)
    N = prm.N
    rng = np.random.default_rng(9)
    u = np.stack([rng.integers(0, mod, size=N, dtype=np.uint64) for mod in basis])
    out = O.moddown(prm, lv, u)
    P = prm.P()
    Q = prm.Q(lv)
    QP = Q * P
    for k in range(N):
        U = _crt(u[:, k], basis)
        Ux = (U + P // 2) % QP                        # round(U/P) = floor((U + floor(P/2))/P), P odd
        got = _crt(out[:, k], prm.q[: lv + 1])
        diff = (got - Ux // P) % Q
        assert diff == 0 or Q - diff < prm.alpha


def test_rescale_is_exact_rounding():
    prm = tiny_params(4, 3, 1)
    lv = prm.L
    N = prm.N
    rng = np.random.default_rng(10)
    c = np.stack([rng.integers(0, q, size=N, dtype=np.uint64) for q in prm.q])
    out = O.rescale_poly(prm, lv, c)
    ql = prm.q[lv]
    Ql = prm.Q(lv)
    for k in range(N):
        U = _crt(c[:, k], prm.q)
        Ux = (U + ql // 2) % Ql
        assert _crt(out[:, k], prm.q[:lv]) == Ux // ql


# --------------------------------------------------------------------------
# encoding
# --------------------------------------------------------------------------
def test_encode_constant_closed_form():
    N = 64
    m = O.encode(np.full(N // 2, 0.75), N, 2.0 ** 20)
    assert m[0] == round(0.75 * 2 ** 20) and not np.any(m[1:])


def test_encode_fft_matches_direct_sum():
    N = 32
    rng = np.random.default_rng(2)
    z = rng.uniform(-1, 1, N // 2)
    assert np.array_equal(O.encode(z, N, 2.0 ** 30), O.encode_direct(z, N, 2.0 ** 30))


def test_decode_encode_roundtrip_and_rotation():
    N = 1 << 12
    rng = np.random.default_rng(4)
    z = rng.uniform(-1, 1, N // 2)
    scale = 2.0 ** 40
    m = O.encode(z, N, scale)
    assert np.max(np.abs(O.decode(m.tolist(), N, scale) - z)) < 2 ** -28
    # decode(phi_5(encode z)) = RotL(z, 1), and phi_{5^-1} gives RotR
    q = Q48
    mm = O.poly_from_signed(m, q)
    for g, shift in ((O.galois_rotl(1, N), -1), (O.galois_rotl(7, N), -7), (O.galois_rotr(3, N), 3)):
        r = O.automorphism(mm, g, q)
        ints = [int(v) if int(v) <= q // 2 else int(v) - q for v in r]
        assert np.max(np.abs(O.decode(ints, N, scale) - np.roll(z, shift))) < 2 ** -28
    # linearity
    z2 = rng.uniform(-1, 1, N // 2)
    assert np.max(np.abs(O.encode(z + z2, N, scale) - O.encode(z, N, scale) - O.encode(z2, N, scale))) <= 2


# --------------------------------------------------------------------------
# encryption, keys, rotations
# --------------------------------------------------------------------------
def test_decrypt_encrypt_error_is_the_sampled_noise():
    prm = tiny_params(6, 3, 1)
    N = prm.N
    s = O.keygen(prm, 77)
    rng = np.random.default_rng(1)
    m = rng.integers(-2 ** 30, 2 ** 30, size=N)
    ct = O.encrypt(prm, s, m, prm.L, seed=99)
    res = O.decrypt(prm, s, ct)
    got = np.array(O.crt_centered(res, prm.q), dtype=object)
    err = got - m
    e = O.sample_cbd21(99, O.stream_enc_e(), N)
    assert np.all(err == e) and max(abs(int(x)) for x in err) <= 21


def test_switching_key_relation():
    prm = tiny_params(5, 3, 2)   # alpha 2 -> 2 digits at level 2
    s = O.keygen(prm, 3)
    g = O.galois_rotl(1, prm.N)
    key = O.rotkey_gen(prm, s, g, 4)
    P = prm.P()
    for j in range(prm.beta(prm.L)):
        e = O.sample_cbd21(4, O.stream_key_e(j, g), prm.N)
        for r, mod in enumerate(prm.qp(prm.L)):
            sr = O.poly_from_signed(s, mod)
            lhs = O.poly_add(key.b[j][r], O.poly_mul_schoolbook(key.a[j][r], sr, mod), mod)
            want = O.poly_from_signed(e, mod)
            if r in prm.digit(prm.L, j):
                want = O.poly_add(want, O.poly_scalar(O.automorphism(sr, g, mod), P % mod, mod), mod)
            assert np.array_equal(lhs, want)


@pytest.mark.parametrize("hoisted", [False, True])
def test_rotation_decrypts_to_rotated_slots(hoisted):
    prm = O.Params.from_dict(W.params_dict("C1"))
    N = prm.N
    s = O.keygen(prm, 21)
    rng = np.random.default_rng(8)
    z = rng.uniform(-1, 1, N // 2)
    m = O.encode(z, N, prm.scale)
    ct = O.encrypt(prm, s, m, prm.L, seed=5)
    for i in (1, 3):
        key = O.rotkey_gen(prm, s, O.galois_rotl(i, N), 6)
        if hoisted:
            rot = O.hoisted_rotate(prm, ct, O.modup(prm, ct.level, ct.c1), key)
        else:
            rot = O.rotate(prm, ct, key)
        dec = O.decrypt_decode(prm, s, rot, prm.scale)
        assert np.max(np.abs(dec - np.roll(z, -i))) < 2 ** -15
        # the error polynomial itself: dec(rot) - phi_g(m) is small
        res = O.decrypt(prm, s, rot)
        got = O.crt_centered(res, prm.q)
        mg = O.automorphism(O.poly_from_signed(m, prm.q[0]), key.g, prm.q[0])
        mg = [int(v) if int(v) <= prm.q[0] // 2 else int(v) - prm.q[0] for v in mg]
        assert max(abs(a - b) for a, b in zip(got, mg)) < 2 ** 12


def test_hoisted_and_unhoisted_differ_only_in_noise():
    prm = tiny_params(5, 2, 1)
    s = O.keygen(prm, 1)
    rng = np.random.default_rng(0)
    m = rng.integers(-2 ** 20, 2 ** 20, size=prm.N)
    ct = O.encrypt(prm, s, m, prm.L, seed=2)
    key = O.rotkey_gen(prm, s, O.galois_rotl(2, prm.N), 3)
    a = O.rotate(prm, ct, key)
    b = O.hoisted_rotate(prm, ct, O.modup(prm, ct.level, ct.c1), key)
    da = np.array(O.crt_centered(O.decrypt(prm, s, a), prm.q), dtype=object)
    db = np.array(O.crt_centered(O.decrypt(prm, s, b), prm.q), dtype=object)
    assert max(abs(int(x)) for x in (da - db)) < 2 ** 10


def test_ct_pt_product_is_exact_negacyclic_product():
    """Rotation-free product: dec(ct * pt) = (m + e) * pt exactly (schoolbook)."""
    prm = tiny_params(4, 2, 1)
    s = O.keygen(prm, 12)
    rng = np.random.default_rng(12)
    m = rng.integers(-2 ** 20, 2 ** 20, size=prm.N)
    pt = rng.integers(-2 ** 10, 2 ** 10, size=prm.N)
    ct = O.encrypt(prm, s, m, prm.L, seed=13)
    out = O.ct_mul_pt(prm, ct, O.reduce_signed(pt, prm.q))
    res = O.decrypt(prm, s, out)
    e = O.sample_cbd21(13, O.stream_enc_e(), prm.N)
    for i, q in enumerate(prm.q):
        want = O.poly_mul_schoolbook(O.poly_from_signed(m + e, q), O.poly_from_signed(pt, q), q)
        assert np.array_equal(res[i], want)


# --------------------------------------------------------------------------
# layouts: the paper's worked examples and complexity tables
# --------------------------------------------------------------------------
def _sym_matrix(m, n):
    """X[r, c] = 100 (r + 1) + c so that symbols can be read back."""
    return np.array([[100.0 * (r + 1) + c for c in range(n)] for r in range(m)])


def _sym(v):
    if v == 0:
        return "0"
    r, c = divmod(int(round(v)), 100)
    return "ABCDEFGH"[r - 1] + str(c)


def test_eq5_worked_example():
    d = json.load(open(os.path.join(GOLD, "paper_examples.json")))
    ex = d["eq5_tall"]
    X = _sym_matrix(ex["m"], ex["n"])
    plan = PL.DiagPlan(ex["m"], ex["n"], slots=4)
    for i, want in ex["diagonals"].items():
        assert [_sym(v) for v in PL.diag_pt_slots(plan, X, int(i))[:4]] == want
    g = d["gala_diag"]
    # GALA's e_i is PackVFL's e_i rotated left by i
    for i, want in g["gala"].items():
        e = PL.diag_pt_slots(plan, X, int(i))[:4]
        assert [_sym(v) for v in np.roll(e, -int(i))] == want
    y = np.array([1000.0, 2000.0])
    assert PL.diag_ct_slots(plan, y)[:4].tolist() == [1000.0, 2000.0, 1000.0, 2000.0]


def test_eq6_worked_example_and_lazy_ras():
    d = json.load(open(os.path.join(GOLD, "paper_examples.json")))
    ex = d["eq6_packing"]
    X = _sym_matrix(ex["m"], ex["n"])
    plan = PL.HybridPlan(ex["m"], ex["n"], ex["slots"])
    assert plan.mprime == ex["mprime"]
    for i, want in ex["diagonals"].items():
        assert [_sym(v) for v in PL.hybrid_pt_slots(plan, X, 0, 0, int(i))] == want
    y = np.array([1.0, 2.0, 3.0, 4.0])
    assert PL.hybrid_ct_slots(plan, y, 0).tolist() == [1.0, 2.0, 3.0, 4.0] * 2
    # lazy RaS: slot contents before the deferred sum, then the final rows
    lz = d["lazy_ras"]
    rng = np.random.default_rng(0)
    Xv = rng.uniform(-1, 1, (4, 4))
    yv = rng.uniform(-1, 1, 4)
    acc = np.zeros(8)
    for i in range(plan.mprime):
        acc += PL.hybrid_pt_slots(plan, Xv, 0, 0, i) * np.roll(PL.hybrid_ct_slots(plan, yv, 0), -i)
    val = lambda sym: Xv["ABCD".index(sym[0]), int(sym[1])] * yv[int(sym[3])]
    for k, terms in enumerate(lz["slots_before_ras"]):
        assert acc[k] == pytest.approx(sum(val(t) for t in terms), abs=1e-15)
    out = PL.hybrid_lazy_ras(plan, [acc])
    for r, terms in enumerate(lz["final"]):
        assert out[r] == pytest.approx(sum(val(t) for t in terms), abs=1e-14)


def test_naive_ras_direction():
    d = json.load(open(os.path.join(GOLD, "paper_examples.json")))["naive_ras"]
    sym = {"A0M0": 3.0, "A1M1": 5.0, "0": 0.0}
    x = np.array([sym[s] for s in d["before"]])
    assert np.roll(x, -1).tolist() == [sym[s] for s in d["after_rotl1"]]


@pytest.mark.parametrize("m,n,S", [(4, 2, 4), (16, 256, 2048), (256, 1024, 4096), (64, 64, 4096),
                                   (100, 37, 64), (8, 2, 4), (32, 8, 8), (8, 32, 8), (32, 32, 8),
                                   (3, 5, 16), (1, 1, 4)])
def test_layout_simulators_equal_matvec(m, n, S):
    rng = np.random.default_rng(m * 1000 + n)
    X = rng.uniform(-1, 1, (m, n))
    y = rng.uniform(-1, 1, n)
    ref = X @ y
    np.testing.assert_allclose(PL.simulate_hybrid(PL.HybridPlan(m, n, S), X, y), ref, atol=1e-12)
    if PL.pow2_ceil(m) <= S and PL.pow2_ceil(n) <= S:
        np.testing.assert_allclose(PL.simulate_diag(PL.DiagPlan(m, n, S, "lazy"), X, y), ref, atol=1e-12)
        np.testing.assert_allclose(PL.simulate_diag(PL.DiagPlan(m, n, S, "rot"), X, y), ref, atol=1e-12)
        np.testing.assert_allclose(PL.simulate_row(PL.RowPlan(m, n, S), X, y), ref, atol=1e-12)


@pytest.mark.parametrize("m,n,nout,S,pack", [(4, 4, 4, 4, 1), (256, 64, 8, 8192, 1), (256, 64, 40, 8192, 32),
                                             (16, 64, 5, 128, 2), (256, 256, 3, 512, 2), (5, 3, 2, 16, 2)])
def test_ctmat_simulator_equals_matmul(m, n, nout, S, pack):
    rng = np.random.default_rng(m + n + nout)
    A = rng.uniform(-1, 1, (m, n))
    Wm = rng.uniform(-1, 1, (n, nout))
    np.testing.assert_allclose(PL.simulate_ctmat(PL.CtMatPlan(m, n, nout, S, pack), A, Wm), A @ Wm, atol=1e-12)


def test_complexity_tables():
    """Table 2 (packvfl row) and Table 3 (with the Table 3 #Add reading for the grid)."""
    import math as _m
    for (m, n, S) in [(64, 64, 4096), (512, 1024, 4096), (256, 1024, 4096), (4096, 4096, 4096)]:
        c = PL.HybridPlan(m, n, S).op_counts()
        k = _m.ceil(m * n / S)
        assert (c["add"], c["mult"], c["rot"], c["hstrot"]) == (k - 1, k, 0, k - 1)
        # Table 2's GALA row: the same terms with O3 rotations instead of hoisted ones
        c = PL.HybridPlan(m, n, S).op_counts(unhoisted=True)
        assert (c["add"], c["mult"], c["rot"], c["hstrot"]) == (k - 1, k, k - 1, 0)
    m, n, S = 64, 8, 8                       # m > N' >= n
    c = PL.HybridPlan(m, n, S).op_counts()
    assert c == {"add": (m * n - m) // S, "mult": m * n // S, "rot": 0, "hstrot": n - 1, "ct_in": 1, "ct_out": m // S}
    m, n, S = 8, 64, 8                       # m <= N' < n
    c = PL.HybridPlan(m, n, S).op_counts()
    assert c == {"add": (n * m - S) // S, "mult": m * n // S, "rot": 0, "hstrot": (m * n - n) // S,
                 "ct_in": n // S, "ct_out": 1}
    m, n, S = 32, 64, 8                      # both > N'
    c = PL.HybridPlan(m, n, S).op_counts()
    assert c == {"add": m * n // S - m // S, "mult": m * n // S, "rot": 0, "hstrot": (n * S - n) // S,
                 "ct_in": n // S, "ct_out": m // S}
    for (m, n) in [(16, 64), (64, 16), (32, 32)]:
        c = PL.DiagPlan(m, n, 256, "rot").op_counts()
        r = int(_m.log2(max(1, n // m)))
        assert (c["add"], c["mult"], c["rot"], c["hstrot"]) == (min(m, n) - 1 + r, min(m, n), r, min(m, n) - 1)
        c = PL.RowPlan(m, n, 256).op_counts()
        assert c["rot"] == m * int(_m.log2(n)) + m - 1 and c["mult"] == 2 * m
