"""Sec. 5.2 in the oracle: Eq. 4 (two products sharing one layout and one
level), the cleartext inverse RaS, and the masked shares of Alg. 2.  CPU only."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import plans as PL
from tests.test_oracle_matmul import tiny


def test_inverse_ras_is_the_papers_split():
    """one round turns [M0, M1] into [M00, M10, M01, M11] with M_i = M_i0 + M_i1"""
    M = np.array([3.25, -1.5])
    u = PL.inverse_ras(M, 1)
    assert u.shape == (4,)
    np.testing.assert_array_equal(u[:2] + u[2:], M)
    np.testing.assert_array_equal(u, [M[0] / 2, M[1] / 2, M[0] / 2, M[1] / 2])
    # k rounds: every part is M_i / 2^k, and summing the 2^k copies restores M exactly
    w = PL.inverse_ras(M, 3)
    np.testing.assert_array_equal(w.reshape(8, 2).sum(axis=0), M)


@pytest.mark.parametrize("m,n,S", [(16, 256, 2048), (100, 37, 64), (64, 8, 16), (8, 64, 16), (3, 5, 8)])
def test_out_slots_survive_the_lazy_ras_hybrid(m, n, S):
    """the lazy RaS (written separately, Sec. 4.3) of the inverse-RaS slots returns v
    (to the rounding of its running sum: the parts are exact, the partial sums k v/2^j need not be)"""
    plan = PL.HybridPlan(m, n, S)
    v = np.random.default_rng(m + n).uniform(-4, 4, m)
    np.testing.assert_allclose(PL.hybrid_lazy_ras(plan, PL.out_slots(plan, v)), v, rtol=0, atol=1e-13)


@pytest.mark.parametrize("m,n", [(16, 64), (64, 16), (5, 37)])
def test_out_slots_survive_the_lazy_ras_diag_and_ctmat(m, n):
    rng = np.random.default_rng(m * n)
    d = PL.DiagPlan(m, n, 128)
    v = rng.uniform(-4, 4, m)
    np.testing.assert_allclose(PL.diag_finish(d, PL.out_slots(d, v)[0]), v, rtol=0, atol=1e-13)
    c = PL.CtMatPlan(m, n, 3, 128 if max(m, n) <= 64 else 256, pack=2)
    V = rng.uniform(-4, 4, (m, 3))
    np.testing.assert_allclose(PL.ctmat_finish(c, PL.out_slots(c, V.ravel())), V, rtol=0, atol=1e-13)


def test_eq4_is_an_identity():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((300, 17))
    z = rng.uniform(-3, 3, 300)
    y = rng.integers(0, 2, 300).astype(float)
    lhs, rhs = PL.eq4_cleartext(0.5, 0.197, -0.004, z, y, X)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kind,m,n", [("hybrid", 8, 32), ("hybrid", 32, 64), ("diag", 4, 16)])
def test_eq4_gradient_with_masked_shares(kind, m, n):
    """g = X^T e by Eq. 4: (q1 X^T)[[z]] + (q2 X^T)[[z^3]] summed over Q u P with
    one ModDown, plus the cleartext (q0 1 - y)^T X through the inverse RaS,
    minus a random slot mask; mask share (lazy RaS of the mask) plus the
    decrypted share equal the cleartext gradient."""
    prm = tiny(6, 2, 1, scale_bits=30)
    N, lv = prm.N, prm.L
    rng = np.random.default_rng(m * 31 + n)
    XB = rng.standard_normal((n, m)) / 4          # batch n x features m; the product takes X^T (m x n)
    z = rng.uniform(-1, 1, n)
    y = rng.integers(0, 2, n).astype(float)
    q0, q1, q2 = 0.5, 0.197, -0.004
    want, _ = PL.eq4_cleartext(q0, q1, q2, z, y, XB)
    XT = XB.T.copy()
    s = O.keygen(prm, 11)
    if kind == "hybrid":
        plan = PL.HybridPlan(m, n, prm.slots)
        gal = PL.hybrid_galois(plan, N)
        ct_ints = lambda v: PL.hybrid_ct_ints(prm, plan, v, prm.scale)  # noqa: E731
        pt_ints = lambda A: PL.hybrid_pt_ints(prm, plan, A, prm.scale)  # noqa: E731
        finish = lambda zs: PL.hybrid_lazy_ras(plan, zs)  # noqa: E731
    else:
        plan = PL.DiagPlan(m, n, prm.slots)
        gal = PL.diag_galois(plan, N)
        ct_ints = lambda v: [O.encode(PL.diag_ct_slots(plan, v), N, prm.scale)]  # noqa: E731
        pt_ints = lambda A: [O.encode(PL.diag_pt_slots(plan, A, i), N, prm.scale) for i in range(plan.ndiag)]  # noqa
        finish = lambda zs: PL.diag_finish(plan, zs[0])  # noqa: E731
    keys = {g: O.rotkey_gen(prm, s, g, 12) for g in gal}
    cz = [O.encrypt(prm, s, mi, lv, 13 + c) for c, mi in enumerate(ct_ints(z))]
    cz3 = [O.encrypt(prm, s, mi, lv, 23 + c) for c, mi in enumerate(ct_ints(z ** 3))]
    outs = PL.hybrid_matmul_sum(prm, plan, [(cz, pt_ints(q1 * XT)), (cz3, pt_ints(q2 * XT))], keys)
    e = int(round(np.log2(prm.scale)))              # output scale Delta^2 = 2^e Delta
    clear = (q0 * np.ones(n) - y) @ XB
    masks = [rng.uniform(-8, 8, prm.slots) for _ in outs]
    shared = []
    for b, ct in enumerate(outs):
        ct = PL.ct_add_plain(prm, ct, PL.encode_at_output(prm, PL.out_slots(plan, clear)[b], lv, e), +1)
        ct = PL.ct_add_plain(prm, ct, PL.encode_at_output(prm, masks[b], lv, e), -1)
        shared.append(O.decrypt_decode(prm, s, ct, prm.scale ** 2))
    share_b = finish(shared)
    share_a = finish(masks)
    got = share_a + share_b
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-4
