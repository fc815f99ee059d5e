"""The oracle's encrypted products decrypt to the plain FP64 definition X y
(or A W) within the precision budget.  CPU only."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import plans as PL
from paper_2405_00482_amd import workloads as W


def rel_err(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def tiny(logN, nq, npr, scale_bits=30, q0_bits=40):
    N = 1 << logN
    out = []
    for bits, cnt in ((q0_bits, 1), (40, nq - 1), (48, npr)):
        x = ((1 << bits) - 1) // (2 * N) * (2 * N) + 1
        got = 0
        while got < cnt:
            if O.is_prime(x) and x not in out:
                out.append(x)
                got += 1
            x -= 2 * N
    return O.Params(logN=logN, q=out[:nq], p=out[nq:], log2_scale=float(scale_bits))


def run_hybrid(prm, X, y, lazy, seed=1, hoisted=True):
    N = prm.N
    plan = PL.HybridPlan(X.shape[0], X.shape[1], prm.slots)
    s = O.keygen(prm, seed)
    keys = {g: O.rotkey_gen(prm, s, g, seed + 1) for g in PL.hybrid_galois(plan, N)}
    cts = [O.encrypt(prm, s, m, prm.L, seed + 2 + c) for c, m in enumerate(PL.hybrid_ct_ints(prm, plan, y, prm.scale))]
    pts = PL.hybrid_pt_ints(prm, plan, X, prm.scale)
    outs = PL.hybrid_matmul(prm, plan, cts, pts, keys, lazy, hoisted)
    zs = [O.decrypt_decode(prm, s, ct, prm.scale * prm.scale) for ct in outs]
    return PL.hybrid_lazy_ras(plan, zs)


@pytest.mark.parametrize("lazy", [True, False])
def test_c1_hybrid_precision(lazy):
    """C1: ring 2^12, Delta 2^30, X^T 16x256 times [[r]]; 2^-20 norm-wise gate for
    the lazy-ModDown plan (the eager plan's extra rounding noise is reported)."""
    prm = O.Params.from_dict(W.params_dict("C1"))
    XT, r = W.c1_inputs()
    got = run_hybrid(prm, XT, r, lazy)
    err = rel_err(got, XT @ r)
    bound = 2.0 ** -20 if lazy else 2.0 ** -18
    assert err < bound, err


@pytest.mark.parametrize("m,n,logN", [(64, 8, 5), (8, 64, 5), (32, 64, 5), (5, 3, 5)])
def test_partitioned_hybrid(m, n, logN):
    prm = tiny(logN, 2, 1)
    rng = np.random.default_rng(m * n)
    X = rng.uniform(-1, 1, (m, n))
    y = rng.uniform(-1, 1, n)
    for lazy in (True, False):
        assert rel_err(run_hybrid(prm, X, y, lazy), X @ y) < 1e-3
    # every rotation a complete O3 rotation (GALA's cost profile, Table 2)
    assert rel_err(run_hybrid(prm, X, y, False, hoisted=False), X @ y) < 1e-3


def test_threaded_evaluation_is_the_serial_one():
    """workers > 1 only spreads independent terms and (output, limb) sums over
    threads: the residues equal the single-threaded evaluation's, here on a
    grid case (two row blocks, two column blocks)"""
    prm = tiny(5, 2, 1)
    N = prm.N
    rng = np.random.default_rng(11)
    X = rng.uniform(-1, 1, (40, 33))
    y = rng.uniform(-1, 1, 33)
    plan = PL.HybridPlan(40, 33, prm.slots)
    assert plan.case == "grid"
    s = O.keygen(prm, 2)
    keys = {g: O.rotkey_gen(prm, s, g, 3) for g in PL.hybrid_galois(plan, N)}
    cts = [O.encrypt(prm, s, m, prm.L, 4 + c) for c, m in enumerate(PL.hybrid_ct_ints(prm, plan, y, prm.scale))]
    pts = PL.hybrid_pt_ints(prm, plan, X, prm.scale)
    one = PL.hybrid_matmul(prm, plan, cts, pts, keys, True)
    many = PL.hybrid_matmul(prm, plan, cts, pts, keys, True, workers=4)
    for a, b in zip(one, many):
        assert np.array_equal(a.c0, b.c0) and np.array_equal(a.c1, b.c1)


def test_c1_hybrid_unhoisted_precision():
    """C1 with O3 rotations: the rotation order changes the bits, not the
    precision class of the per-rotation ModDown plan."""
    prm = O.Params.from_dict(W.params_dict("C1"))
    XT, r = W.c1_inputs()
    assert rel_err(run_hybrid(prm, XT, r, False, hoisted=False), XT @ r) < 2.0 ** -18


@pytest.mark.parametrize("m,n", [(16, 4), (4, 16)])
def test_diag_plan(m, n):
    prm = tiny(5, 2, 1)
    N = prm.N
    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, (m, n))
    y = rng.uniform(-1, 1, n)
    s = O.keygen(prm, 4)
    for ras in ("lazy", "rot"):
        plan = PL.DiagPlan(m, n, prm.slots, ras)
        keys = {g: O.rotkey_gen(prm, s, g, 5) for g in PL.diag_galois(plan, N)}
        ct = O.encrypt(prm, s, O.encode(PL.diag_ct_slots(plan, y), N, prm.scale), prm.L, 6)
        pts = [O.encode(PL.diag_pt_slots(plan, X, i), N, prm.scale) for i in range(plan.ndiag)]
        for hoisted in (True, False):
            out = PL.diag_matmul(prm, plan, ct, pts, keys, lazy=False, hoisted=hoisted)
            z = O.decrypt_decode(prm, s, out, prm.scale ** 2)
            assert rel_err(PL.diag_finish(plan, z), X @ y) < 1e-3


def test_row_plan_two_rescales():
    prm = tiny(5, 3, 1, scale_bits=30, q0_bits=45)
    N = prm.N
    rng = np.random.default_rng(4)
    m, n = 6, 8
    X = rng.uniform(-1, 1, (m, n))
    y = rng.uniform(-1, 1, n)
    plan = PL.RowPlan(m, n, prm.slots)
    s = O.keygen(prm, 7)
    keys = {g: O.rotkey_gen(prm, s, g, 8) for g in PL.row_galois(plan, N)}
    ct_slots = np.zeros(prm.slots)
    for t in range(prm.slots):
        ct_slots[t] = y[t % plan.np_] if t % plan.np_ < n else 0.0
    ct = O.encrypt(prm, s, O.encode(ct_slots, N, prm.scale), prm.L, 9)
    pts = [O.encode(PL.row_pt_slots(plan, X, r), N, prm.scale) for r in range(m)]
    ind = np.zeros(prm.slots)
    ind[0] = 1.0
    ind_ints = O.encode(ind, N, float(prm.q[1]))
    out = PL.row_matmul(prm, plan, ct, pts, ind_ints, keys)
    assert out.level == 0
    z = O.decrypt_decode(prm, s, out, prm.scale ** 2 / prm.q[2])
    assert rel_err(z[:m], X @ y) < 1e-3


@pytest.mark.parametrize("pack", [1, 2])
def test_ctmat_plan(pack):
    prm = tiny(5, 2, 1)
    N = prm.N
    rng = np.random.default_rng(5)
    A = rng.uniform(-1, 1, (8, 4))
    Wm = rng.normal(0, 0.1, (4, 3))
    plan = PL.CtMatPlan(8, 4, 3, prm.slots, pack)
    s = O.keygen(prm, 2)
    cts = [O.encrypt(prm, s, O.encode(PL.ctmat_ct_slots(plan, A, i), N, prm.scale), prm.L, 30 + i)
           for i in range(plan.ndiag)]
    pts = [O.encode(PL.ctmat_pt_slots(plan, Wm, i, k), N, prm.scale)
           for i in range(plan.ndiag) for k in range(plan.n_out_cts)]
    outs = PL.ctmat_matmul(prm, plan, cts, pts)
    zs = [O.decrypt_decode(prm, s, c, prm.scale ** 2) for c in outs]
    assert rel_err(PL.ctmat_finish(plan, zs), A @ Wm) < 1e-3


@pytest.mark.parametrize("m,n,S,bs", [(64, 64, 64, 2), (64, 64, 64, 8), (32, 128, 64, 4), (200, 300, 64, 2),
                                      (16, 256, 64, 8)])
def test_bsgs_reorder_is_exact_in_cleartext(m, n, S, bs):
    """The baby-step/giant-step regrouping computes X y exactly as the
    hoisted diagonal sum does (cleartext slots, FP64)."""
    plan = PL.HybridPlan(m, n, S)
    if not PL.bsgs_valid(plan, bs):
        pytest.skip("m' too small for this baby step")
    rng = np.random.default_rng(m + n + bs)
    X = rng.uniform(-1, 1, (m, n))
    y = rng.uniform(-1, 1, n)
    got = PL.simulate_hybrid_bsgs(plan, X, y, bs)
    assert np.allclose(got, X @ y, rtol=0, atol=1e-11)
    assert np.allclose(got, PL.simulate_hybrid(plan, X, y), rtol=0, atol=1e-11)


def test_bsgs_galois_set():
    plan = PL.HybridPlan(64, 64, 64)      # m' = 64
    gs = PL.bsgs_galois(plan, 128, 8)
    want = {O.galois_rotl(k, 128) for k in range(1, 8)} | {O.galois_rotl(8 * j, 128) for j in range(1, 8)}
    assert set(gs) == want and len(gs) == 14


@pytest.mark.parametrize("m,n,bs", [(32, 32, 4), (64, 16, 2), (8, 64, 2)])
def test_bsgs_encrypted(m, n, bs):
    prm = tiny(6, 2, 1)
    N = prm.N
    plan = PL.HybridPlan(m, n, prm.slots)
    assert PL.bsgs_valid(plan, bs)
    rng = np.random.default_rng(9)
    X = rng.uniform(-1, 1, (m, n))
    y = rng.uniform(-1, 1, n)
    s = O.keygen(prm, 11)
    keys = {g: O.rotkey_gen(prm, s, g, 12) for g in PL.bsgs_galois(plan, N, bs)}
    cts = [O.encrypt(prm, s, mm, prm.L, 13 + c) for c, mm in enumerate(PL.hybrid_ct_ints(prm, plan, y, prm.scale))]
    pts = PL.bsgs_pt_ints(prm, plan, X, prm.scale, bs)
    outs = PL.hybrid_matmul_bsgs(prm, plan, cts, pts, keys, bs)
    zs = [O.decrypt_decode(prm, s, ct, prm.scale * prm.scale) for ct in outs]
    assert rel_err(PL.hybrid_lazy_ras(plan, zs), X @ y) < 1e-3


@pytest.mark.parametrize("m,n", [(4, 4), (8, 2), (2, 8), (16, 4), (4, 16), (3, 5), (7, 3), (64, 16), (1, 8)])
def test_transpose_conversion_is_a_slot_permutation(m, n):
    """Eq. 7 (reading): rotating A's diagonals gives exactly A^T's diagonals
    (cleartext slots, fully replicated layout)."""
    S = 128
    rng = np.random.default_rng(m * 31 + n)
    A = rng.uniform(-1, 1, (m, n))
    width = max(PL.pow2_ceil(m), PL.pow2_ceil(n))
    plan = PL.CtMatPlan(m, n, 1, S, pack=S // width)
    planT = PL.CtMatPlan(n, m, 1, S, pack=S // width)
    e = [PL.ctmat_ct_slots(plan, A, i) for i in range(plan.ndiag)]
    for i, (k, r) in enumerate(PL.transpose_map(plan)):
        assert np.array_equal(np.roll(e[k], -r), PL.ctmat_ct_slots(planT, A.T, i)), (i, k, r)


def test_transpose_conversion_as_printed_fails():
    """the literal Eq. 7 does not give A^T's diagonals for a tall matrix"""
    S = 64
    A = np.arange(1, 33, dtype=float).reshape(8, 4)
    plan = PL.CtMatPlan(8, 4, 1, S, pack=S // 8)
    planT = PL.CtMatPlan(4, 8, 1, S, pack=S // 8)
    e = [PL.ctmat_ct_slots(plan, A, i) for i in range(plan.ndiag)]
    ok = [np.array_equal(np.roll(e[k], -r), PL.ctmat_ct_slots(planT, A.T, i))
          for i, (k, r) in enumerate(PL.transpose_map_as_printed(plan))]
    assert not all(ok)


@pytest.mark.parametrize("m,n", [(8, 4), (4, 8)])
def test_transpose_then_backward_product_encrypted(m, n):
    """[[A]] -> [[A^T]] by Eq. 7, then Alg. 3 with B: decrypts to A^T B."""
    prm = tiny(6, 2, 1)
    N, S = prm.N, prm.slots
    rng = np.random.default_rng(5)
    A = rng.uniform(-1, 1, (m, n))
    B = rng.uniform(-1, 1, (m, 3))
    width = max(m, n)
    plan = PL.CtMatPlan(m, n, 1, S, pack=S // width)
    planT = PL.CtMatPlan(n, m, 3, S, pack=S // width)
    s = O.keygen(prm, 21)
    keys = {g: O.rotkey_gen(prm, s, g, 22) for g in PL.transpose_galois(plan, N)}
    cts = [O.encrypt(prm, s, O.encode(PL.ctmat_ct_slots(plan, A, i), N, prm.scale), prm.L, 23 + i)
           for i in range(plan.ndiag)]
    ctsT = PL.ctmat_transpose(prm, plan, cts, keys)
    pts = [O.encode(PL.ctmat_pt_slots(planT, B, i, k), N, prm.scale)
           for i in range(planT.ndiag) for k in range(planT.n_out_cts)]
    outs = PL.ctmat_matmul(prm, planT, ctsT, pts)
    zs = [O.decrypt_decode(prm, s, ct, prm.scale ** 2) for ct in outs]
    got = PL.ctmat_finish(planT, zs)
    assert rel_err(got, A.T @ B) < 1e-3


@pytest.mark.parametrize("m,n", [(16, 8), (100, 5), (64, 3)])
def test_column_order_plan(m, n):
    """Sec. 3.1's column-order method: the layout simulator is X y, Table 2's
    counts hold, and the encrypted product decrypts to X y"""
    prm = tiny(5, 2, 1)
    N = prm.N
    rng = np.random.default_rng(m + n)
    X = rng.uniform(-1, 1, (m, n))
    y = rng.uniform(-1, 1, n)
    plan = PL.ColPlan(m, n, prm.slots)
    np.testing.assert_allclose(PL.simulate_col(plan, X, y), X @ y, atol=1e-12)
    c = plan.op_counts()
    assert (c["mult"], c["add"], c["rot"], c["hstrot"], c["ct_in"]) == (
        n * plan.row_blocks, (n - 1) * plan.row_blocks, 0, 0, n)
    s = O.keygen(prm, 4)
    cts = [O.encrypt(prm, s, O.encode(PL.col_ct_slots(plan, y, j), N, prm.scale), prm.L, 10 + j) for j in range(n)]
    outs = PL.col_matmul(prm, plan, cts, PL.col_pt_ints(prm, plan, X, prm.scale))
    zs = [O.decrypt_decode(prm, s, ct, prm.scale ** 2) for ct in outs]
    assert rel_err(PL.col_finish(plan, zs), X @ y) < 1e-3
