"""Packing plans of PackVFL as plain index maps plus their evaluation on the
oracle scheme.  TEST INFRASTRUCTURE ONLY (see oracle.py).

A plan maps a real m x n matrix X and a real vector y (or an encrypted matrix A
and a plaintext W) onto slot vectors.  Every layout here is written straight
from the paper's equations:

* diagonal encoding, Eq. 5:  e_i[j] = X[j mod m, (i+j) mod n];
* input packing, Eq. 6:      X'[i mod m', j + n*floor(i/m')] = X[i, j],
  m' = ceil(m n / N'), then Eq. 5 applied per n-wide part of X' (Sec. 4.2:
  "diagonal encoding is performed in parts"), i.e.
      e_i[g n + j] = X[g m' + (j mod m'), (i + j) mod n],  i < m', g < N'/n;
* the encrypted vector replicated with period n over all N' slots (Sec. 4.1);
* input partitioning (Sec. 4.2): row blocks of N' rows sharing one set of
  hoisted rotations when m > N' >= n, column blocks (and input ciphertexts)
  added before sending when m <= N' < n, both when both exceed N';
* lazy rotate-and-sum (Sec. 4.3): after decryption,
      out[g m' + r] = sum_{t < n/m'} z[g n + r + t m'];
* row-order (naive) method (Sec. 3.1): per row, Mult, log2 n RaS rotations,
  indicator mask, placement rotation;
* ciphertext-matrix times plaintext-matrix (Alg. 3): the encrypted matrix
  is sent as its Eq. 5 diagonals and each output column is
  sum_i [[e_i]] * w_i with w_i[j] = W[(i+j) mod n, k], no rotations.

Readings where the paper is silent or garbled: m and n are zero-padded to
powers of two (Sec. 3 says so), and m' is rounded up to a power of two so
that m' divides n (needed for the lazy RaS sum to close).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import oracle as O


def pow2_ceil(x: int) -> int:
    p = 1
    while p < x:
        p <<= 1
    return p


# ---------------------------------------------------------------------------
# plan descriptions
# ---------------------------------------------------------------------------
@dataclass
class HybridPlan:
    """X (m x n, plaintext) times [[y]] (n, encrypted): the PackVFL hybrid."""
    m: int
    n: int
    slots: int
    mp: int = 0          # padded m
    np_: int = 0         # padded n
    case: str = ""       # "S", "row", "col", "grid"
    row_blocks: int = 1  # output ciphertexts
    col_blocks: int = 1  # input ciphertexts
    bm: int = 0          # rows per block (padded)
    bn: int = 0          # columns per block (padded)
    mprime: int = 0      # diagonals per block (m')
    G: int = 0           # groups per ciphertext (N' / bn)

    def __post_init__(self):
        S = self.slots
        self.mp = pow2_ceil(self.m)
        self.np_ = pow2_ceil(self.n)
        self.row_blocks = max(1, self.mp // S)
        self.col_blocks = max(1, self.np_ // S)
        self.bm = min(self.mp, S)
        self.bn = min(self.np_, S)
        self.case = {(1, 1): "S", (2, 1): "row", (1, 2): "col", (2, 2): "grid"}[
            (1 + (self.row_blocks > 1), 1 + (self.col_blocks > 1))]
        self.mprime = max(1, (self.bm * self.bn) // S)
        self.G = S // self.bn

    @property
    def rotations(self) -> list:
        """rotation amounts of the hoisted set (0 = unrotated term)"""
        return list(range(self.mprime))

    def terms(self):
        """(in_ct, rot, pt_index, out_ct) of every pt x rotated-ct product"""
        out = []
        for b in range(self.row_blocks):
            for c in range(self.col_blocks):
                for i in range(self.mprime):
                    out.append((c, i, (b * self.col_blocks + c) * self.mprime + i, b))
        return out

    @property
    def n_pts(self) -> int:
        return self.row_blocks * self.col_blocks * self.mprime

    def op_counts(self, unhoisted: bool = False) -> dict:
        """Tables 2 and 3 counts of this plan (lazy RaS: no O3).  unhoisted:
        every diagonal rotation a complete O3 rotation of its input ciphertext,
        once per (row block, column block) term -- Table 2's GALA row."""
        mults = self.n_pts
        adds = mults - self.row_blocks
        if unhoisted:
            rot = self.row_blocks * self.col_blocks * (self.mprime - 1)
            return {"add": adds, "mult": mults, "rot": rot, "hstrot": 0,
                    "ct_in": self.col_blocks, "ct_out": self.row_blocks}
        hst = self.col_blocks * (self.mprime - 1)
        return {"add": adds, "mult": mults, "rot": 0, "hstrot": hst,
                "ct_in": self.col_blocks, "ct_out": self.row_blocks}


def hybrid_pt_slots(plan: HybridPlan, X: np.ndarray, b: int, c: int, i: int) -> np.ndarray:
    """Slot vector of diagonal i of block (b, c): blockwise Eq. 5 on Eq. 6's X'."""
    S = plan.slots
    z = np.zeros(S, dtype=np.float64)
    m, n = X.shape
    for g in range(plan.G):
        for j in range(plan.bn):
            row = b * plan.bm + g * plan.mprime + (j % plan.mprime)
            col = c * plan.bn + (i + j) % plan.bn
            if row < m and col < n and g * plan.mprime + (j % plan.mprime) < plan.bm:
                z[g * plan.bn + j] = X[row, col]
    return z


def hybrid_ct_slots(plan: HybridPlan, y: np.ndarray, c: int) -> np.ndarray:
    """Input ciphertext c: column block c of y replicated with period bn."""
    S = plan.slots
    z = np.zeros(S, dtype=np.float64)
    for t in range(S):
        col = c * plan.bn + (t % plan.bn)
        if col < y.size:
            z[t] = y[col]
    return z


def hybrid_lazy_ras(plan: HybridPlan, zs: list) -> np.ndarray:
    """Sec. 4.3: out[b N' + g m' + r] = sum_t z_b[g bn + r + t m'] (cleartext)."""
    out = np.zeros(plan.m, dtype=np.float64)
    for b in range(plan.row_blocks):
        z = zs[b]
        for g in range(plan.G):
            for r in range(plan.mprime):
                row = b * plan.bm + g * plan.mprime + r
                if row >= plan.m or g * plan.mprime + r >= plan.bm:
                    continue
                out[row] = sum(z[g * plan.bn + r + t * plan.mprime] for t in range(plan.bn // plan.mprime))
    return out


def simulate_hybrid(plan: HybridPlan, X, y) -> np.ndarray:
    """Cleartext FP64 run of the plan's slot arithmetic (no encryption)."""
    S = plan.slots
    cts = [hybrid_ct_slots(plan, y, c) for c in range(plan.col_blocks)]
    acc = [np.zeros(S) for _ in range(plan.row_blocks)]
    for (c, i, k, b) in plan.terms():
        bb, cc, ii = k // (plan.col_blocks * plan.mprime), (k // plan.mprime) % plan.col_blocks, k % plan.mprime
        assert (bb, cc, ii) == (b, c, i)
        acc[b] += hybrid_pt_slots(plan, X, b, c, i) * np.roll(cts[c], -i)
    return hybrid_lazy_ras(plan, acc)


@dataclass
class DiagPlan:
    """Eq. 5 verbatim: min(m,n) diagonals over max(m,n) slots, no input packing."""
    m: int
    n: int
    slots: int
    ras: str = "lazy"     # "lazy" or "rot" (in-ciphertext RaS by RotL(m 2^k))

    def __post_init__(self):
        self.mp = pow2_ceil(self.m)
        self.np_ = pow2_ceil(self.n)
        assert self.mp <= self.slots and self.np_ <= self.slots, "DIAG has no partitioning"
        self.ndiag = min(self.mp, self.np_)
        self.width = max(self.mp, self.np_)

    def ras_rotations(self) -> list:
        if self.mp >= self.np_ or self.ras == "lazy":
            return []
        out, k = [], self.mp
        while k < self.np_:
            out.append(k)
            k *= 2
        return out

    def op_counts(self) -> dict:
        r = len(self.ras_rotations())
        return {"add": self.ndiag - 1 + r, "mult": self.ndiag, "rot": r, "hstrot": self.ndiag - 1,
                "ct_in": 1, "ct_out": 1}


def diag_pt_slots(plan: DiagPlan, X, i) -> np.ndarray:
    z = np.zeros(plan.slots)
    m, n = X.shape
    for j in range(plan.width):
        r, c = j % plan.mp, (i + j) % plan.np_
        if r < m and c < n:
            z[j] = X[r, c]
    return z


def diag_ct_slots(plan: DiagPlan, y) -> np.ndarray:
    z = np.zeros(plan.slots)
    for t in range(plan.slots):
        if t % plan.np_ < y.size:
            z[t] = y[t % plan.np_]
    return z


def diag_finish(plan: DiagPlan, z) -> np.ndarray:
    """Read rows from the decrypted slots: directly if m >= n or the RaS ran in
    the ciphertext, else the lazy RaS sum over n/m slot groups."""
    out = np.zeros(plan.m)
    for r in range(plan.m):
        if plan.mp >= plan.np_ or plan.ras == "rot":
            out[r] = z[r]
        else:
            out[r] = sum(z[r + t * plan.mp] for t in range(plan.np_ // plan.mp))
    return out


def simulate_diag(plan: DiagPlan, X, y) -> np.ndarray:
    ct = diag_ct_slots(plan, y)
    acc = np.zeros(plan.slots)
    for i in range(plan.ndiag):
        acc += diag_pt_slots(plan, X, i) * np.roll(ct, -i)
    for k in plan.ras_rotations():
        acc = acc + np.roll(acc, -k)
    return diag_finish(plan, acc)


@dataclass
class RowPlan:
    """Sec. 3.1 row-order method: m log2 n + m - 1 rotations, 2m mults."""
    m: int
    n: int
    slots: int

    def __post_init__(self):
        self.mp = pow2_ceil(self.m)
        self.np_ = pow2_ceil(self.n)
        assert self.np_ <= self.slots and self.m <= self.slots
        self.log_n = self.np_.bit_length() - 1

    def ras_rotations(self) -> list:
        return [1 << k for k in range(self.log_n)]

    def op_counts(self) -> dict:
        m = self.m
        return {"add": m * self.log_n + m - 1, "mult": 2 * m, "rot": m * self.log_n + m - 1,
                "hstrot": 0, "ct_in": 1, "ct_out": 1}


def row_pt_slots(plan: RowPlan, X, r) -> np.ndarray:
    z = np.zeros(plan.slots)
    z[: X.shape[1]] = X[r]
    return z


def simulate_row(plan: RowPlan, X, y) -> np.ndarray:
    ct = np.zeros(plan.slots)
    for t in range(plan.slots):
        if t % plan.np_ < y.size:
            ct[t] = y[t % plan.np_]
    acc = np.zeros(plan.slots)
    ind = np.zeros(plan.slots)
    ind[0] = 1.0
    for r in range(plan.m):
        t = row_pt_slots(plan, X, r) * ct
        for k in plan.ras_rotations():
            t = t + np.roll(t, -k)
        t = t * ind
        acc += np.roll(t, r)
    return acc[: plan.m]


@dataclass
class ColPlan:
    """Sec. 3.1 column-order method: plaintext j holds column j of X, input
    ciphertext j holds y_j in every slot; out = sum_j pt_j * ct_j, no rotation.
    m > N' takes row blocks of N' rows (one output ciphertext each)."""
    m: int
    n: int
    slots: int

    def __post_init__(self):
        self.mp = pow2_ceil(self.m)
        self.bm = min(self.mp, self.slots)
        self.row_blocks = max(1, -(-self.mp // self.slots))

    def op_counts(self) -> dict:
        rb = self.row_blocks
        return {"add": (self.n - 1) * rb, "mult": self.n * rb, "rot": 0, "hstrot": 0, "ct_in": self.n, "ct_out": rb}


def col_pt_slots(plan: ColPlan, X, j: int, b: int) -> np.ndarray:
    z = np.zeros(plan.slots)
    rows = X[b * plan.bm:(b + 1) * plan.bm, j]
    z[: rows.size] = rows
    return z


def col_ct_slots(plan: ColPlan, y, j: int) -> np.ndarray:
    return np.full(plan.slots, float(y[j]))


def col_finish(plan: ColPlan, zs) -> np.ndarray:
    return np.array([zs[r // plan.bm][r % plan.bm] for r in range(plan.m)])


def simulate_col(plan: ColPlan, X, y) -> np.ndarray:
    zs = [sum(col_pt_slots(plan, X, j, b) * col_ct_slots(plan, y, j) for j in range(plan.n))
          for b in range(plan.row_blocks)]
    return col_finish(plan, zs)


@dataclass
class CtMatPlan:
    """Alg. 3: [[A]] (m x n, encrypted as Eq. 5 diagonals) times W (n x n').

    pack = columns of W per plaintext (1 = one output ciphertext per column,
    as in Alg. 3; up to N'/max(m,n) by replicating each diagonal ciphertext).
    """
    m: int
    n: int
    nout: int
    slots: int
    pack: int = 1

    def __post_init__(self):
        self.mp = pow2_ceil(self.m)
        self.np_ = pow2_ceil(self.n)
        self.width = max(self.mp, self.np_)
        assert self.width <= self.slots
        assert self.pack >= 1 and self.pack * self.width <= self.slots
        self.ndiag = min(self.mp, self.np_)
        self.n_out_cts = -(-self.nout // self.pack)

    @property
    def n_pts(self) -> int:
        return self.ndiag * self.n_out_cts

    def op_counts(self) -> dict:
        return {"add": self.n_pts - self.n_out_cts, "mult": self.n_pts, "rot": 0, "hstrot": 0,
                "ct_in": self.ndiag, "ct_out": self.n_out_cts}


def ctmat_ct_slots(plan: CtMatPlan, A, i) -> np.ndarray:
    """Diagonal i of A (Eq. 5), replicated over `pack` blocks of width max(m,n)."""
    z = np.zeros(plan.slots)
    m, n = A.shape
    for b in range(plan.pack):
        for j in range(plan.width):
            r, c = j % plan.mp, (i + j) % plan.np_
            if r < m and c < n:
                z[b * plan.width + j] = A[r, c]
    return z


def ctmat_pt_slots(plan: CtMatPlan, W, i, k) -> np.ndarray:
    """Plaintext for diagonal i and output ciphertext k: w[b W + j] = W[(i+j) mod n, k pack + b]."""
    z = np.zeros(plan.slots)
    n, nout = W.shape
    for b in range(plan.pack):
        col = k * plan.pack + b
        if col >= nout:
            continue
        for j in range(plan.width):
            r = (i + j) % plan.np_
            if r < n:
                z[b * plan.width + j] = W[r, col]
    return z


def ctmat_finish(plan: CtMatPlan, zs) -> np.ndarray:
    out = np.zeros((plan.m, plan.nout))
    for k, z in enumerate(zs):
        for b in range(plan.pack):
            col = k * plan.pack + b
            if col >= plan.nout:
                continue
            for r in range(plan.m):
                if plan.mp >= plan.np_:
                    out[r, col] = z[b * plan.width + r]
                else:
                    out[r, col] = sum(z[b * plan.width + r + t * plan.mp] for t in range(plan.np_ // plan.mp))
    return out


def simulate_ctmat(plan: CtMatPlan, A, W) -> np.ndarray:
    cts = [ctmat_ct_slots(plan, A, i) for i in range(plan.ndiag)]
    zs = []
    for k in range(plan.n_out_cts):
        acc = np.zeros(plan.slots)
        for i in range(plan.ndiag):
            acc += cts[i] * ctmat_pt_slots(plan, W, i, k)
        zs.append(acc)
    return ctmat_finish(plan, zs)


# ---------------------------------------------------------------------------
# homomorphic evaluation of the plans on the oracle scheme
# ---------------------------------------------------------------------------
def encode_residues(params: O.Params, slots_vec, scale: float, primes) -> np.ndarray:
    m = O.encode(slots_vec, params.N, scale)
    return O.reduce_signed(m, primes)


def hybrid_matmul(params: O.Params, plan, cts, pt_ints, keys: dict, lazy: bool, hoisted: bool = True,
                  workers: int = 1) -> list:
    """Evaluate the hybrid plan (or any plan given as `terms()`).

    cts: input ciphertexts (coefficient domain); pt_ints: integer coefficient
    vectors (int64[N]) of every diagonal plaintext, indexed as in terms();
    keys: Galois element -> SwitchKey.  Returns the output ciphertexts.

    eager (paper-literal, Alg. 1): out = sum_i pt_i * HstRotL(ct, i), each hoisted
      rotation finished by its own ModDown;
    lazy: acc = sum_i pt_i^{QP} * (P*phi_i(c0) + u0_i, u1_i) over Q u P and one
      ModDown per output (the i = 0 term uses (P*c0, P*c1)).
    hoisted = False (eager only): every rotation a complete O3 rotation
      (automorphism, then its own ModUp; Sec. 2), once per term -- the cost
      profile of GALA's method (Table 2).
    workers > 1 (lazy only): the independent rotated terms, and the
      accumulation of each (output, limb) pair, run on that many threads (the
      C core releases the interpreter lock); every sum still takes the terms
      in terms() order, so the residues are the same as with one worker.
    """
    assert hoisted or not lazy, "unhoisted rotations are evaluated with per-rotation ModDown"
    N = params.N
    lv = cts[0].level
    Qp = params.q[: lv + 1]
    QPp = params.qp(lv)
    Pint = params.P()
    terms = plan.terms()
    n_out = max(t[3] for t in terms) + 1
    digits = {}
    if hoisted:
        for c in set(t[0] for t in terms):
            digits[c] = O.modup(params, lv, cts[c].c1)
    if not lazy:
        outs = [O.zero_ct(params, lv) for _ in range(n_out)]
        rot_cache = {}
        for (c, i, k, b) in terms:
            if (c, i) not in rot_cache:
                if i == 0:
                    rot_cache[(c, i)] = cts[c]
                elif hoisted:
                    g = O.galois_rotl(i, N)
                    rot_cache[(c, i)] = O.hoisted_rotate(params, cts[c], digits[c], keys[g])
                else:
                    rot_cache[(c, i)] = O.rotate(params, cts[c], keys[O.galois_rotl(i, N)])
            pt = O.reduce_signed(pt_ints[k], Qp)
            outs[b] = O.ct_add(params, outs[b], O.ct_mul_pt(params, rot_cache[(c, i)], pt))
        return outs
    acc0 = [np.zeros((len(QPp), N), dtype=np.uint64) for _ in range(n_out)]
    acc1 = [np.zeros((len(QPp), N), dtype=np.uint64) for _ in range(n_out)]
    pairs = list(dict.fromkeys((c, i) for (c, i, k, b) in terms))
    term_cache = dict(zip(pairs, _pmap(lambda ci: lazy_term(params, cts[ci[0]], digits[ci[0]], keys, ci[1]),
                                       pairs, workers)))

    def accumulate(br):
        b, r = br
        mod = QPp[r]
        for (c, i, k, bb) in terms:
            if bb != b:
                continue
            t0, t1 = term_cache[(c, i)]
            pt = O.reduce_signed(pt_ints[k], [mod])[0]
            acc0[b][r] = O.poly_add(acc0[b][r], O.poly_mul(pt, t0[r], mod), mod)
            acc1[b][r] = O.poly_add(acc1[b][r], O.poly_mul(pt, t1[r], mod), mod)

    _pmap(accumulate, [(b, r) for b in range(n_out) for r in range(len(QPp))], workers)
    return [O.Ciphertext(O.moddown(params, lv, acc0[b]), O.moddown(params, lv, acc1[b]), lv)
            for b in range(n_out)]


def _pmap(fn, items, workers: int) -> list:
    """[fn(x) for x in items], on `workers` threads when workers > 1"""
    if workers <= 1:
        return [fn(x) for x in items]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(fn, items))


def lazy_term(params: O.Params, ct, digits, keys: dict, i: int):
    """RotL(ct, i) over Q u P before its ModDown: (P*phi(c0) + u0, u1) with
    (u0, u1) the key inner product of phi(digits); i = 0 gives (P*c0, P*c1)."""
    N = params.N
    lv = ct.level
    Qp = params.q[: lv + 1]
    QPp = params.qp(lv)
    Pint = params.P()
    if i == 0:
        t0 = np.zeros((len(QPp), N), dtype=np.uint64)
        t1 = np.zeros_like(t0)
        for r in range(lv + 1):
            t0[r] = O.poly_scalar(ct.c0[r], Pint % Qp[r], Qp[r])
            t1[r] = O.poly_scalar(ct.c1[r], Pint % Qp[r], Qp[r])
        return t0, t1
    g = O.galois_rotl(i, N)
    u0, u1 = O.inner_product(params, lv, digits, keys[g], g)
    c0r = O.automorphism_ct_part(params, lv, ct.c0, g)
    for r in range(lv + 1):
        u0[r] = O.poly_add(u0[r], O.poly_scalar(c0r[r], Pint % Qp[r], Qp[r]), Qp[r])
    return u0, u1


def hybrid_pt_ints(params: O.Params, plan: HybridPlan, X, scale: float) -> list:
    out = []
    for b in range(plan.row_blocks):
        for c in range(plan.col_blocks):
            for i in range(plan.mprime):
                out.append(O.encode(hybrid_pt_slots(plan, X, b, c, i), params.N, scale))
    return out


def hybrid_ct_ints(params: O.Params, plan: HybridPlan, y, scale: float) -> list:
    return [O.encode(hybrid_ct_slots(plan, y, c), params.N, scale) for c in range(plan.col_blocks)]


def hybrid_galois(plan, N: int) -> list:
    return [O.galois_rotl(i, N) for i in range(1, plan.mprime)]


# ---------------------------------------------------------------------------
# baby-step/giant-step schedule of the hybrid's diagonal sum (Halevi-Shoup
# 2018; not in the paper, one of the rotation schedules the planner weighs).
# With diagonal i = j*bs + k (k < bs, j < g = m'/bs):
#     sum_i pt_i * RotL(ct, i) = sum_j RotL( sum_k RotL(pt_i, -j*bs) * RotL(ct, k), j*bs )
# The bs - 1 baby rotations share one ModUp and stay over Q u P (as in the
# lazy hoisted form); every inner sum is brought down to Q by its own ModDown
# and, for j > 0, rotated by j*bs with its own key switch (ModUp of the
# sum's c1, phi on the digits, ModDown).
# ---------------------------------------------------------------------------
def bsgs_valid(plan: HybridPlan, bs: int) -> bool:
    return bs >= 2 and (bs & (bs - 1)) == 0 and 2 * bs <= plan.mprime


def bsgs_pt_slots(plan: HybridPlan, X, b: int, c: int, i: int, bs: int) -> np.ndarray:
    """diagonal i pre-rotated right by its giant step: RotL(pt_i, -(i // bs) * bs)"""
    return np.roll(hybrid_pt_slots(plan, X, b, c, i), (i // bs) * bs)


def bsgs_pt_ints(params: O.Params, plan: HybridPlan, X, scale: float, bs: int) -> list:
    out = []
    for b in range(plan.row_blocks):
        for c in range(plan.col_blocks):
            for i in range(plan.mprime):
                out.append(O.encode(bsgs_pt_slots(plan, X, b, c, i, bs), params.N, scale))
    return out


def bsgs_galois(plan: HybridPlan, N: int, bs: int) -> list:
    g = plan.mprime // bs
    gs = [O.galois_rotl(k, N) for k in range(1, bs)] + [O.galois_rotl(j * bs, N) for j in range(1, g)]
    return sorted(set(gs))


def simulate_hybrid_bsgs(plan: HybridPlan, X, y, bs: int) -> np.ndarray:
    """Cleartext FP64 run of the baby-step/giant-step evaluation order."""
    S = plan.slots
    g = plan.mprime // bs
    cts = [hybrid_ct_slots(plan, y, c) for c in range(plan.col_blocks)]
    acc = [np.zeros(S) for _ in range(plan.row_blocks)]
    for b in range(plan.row_blocks):
        for c in range(plan.col_blocks):
            for j in range(g):
                inner = np.zeros(S)
                for k in range(bs):
                    inner += bsgs_pt_slots(plan, X, b, c, j * bs + k, bs) * np.roll(cts[c], -k)
                acc[b] += np.roll(inner, -j * bs)
    return hybrid_lazy_ras(plan, acc)


def hybrid_matmul_bsgs(params: O.Params, plan: HybridPlan, cts, pt_ints, keys: dict, bs: int) -> list:
    """Evaluate the hybrid plan in baby-step/giant-step order; pt_ints from
    bsgs_pt_ints (pre-rotated diagonals)."""
    assert bsgs_valid(plan, bs)
    N = params.N
    lv = cts[0].level
    QPp = params.qp(lv)
    g = plan.mprime // bs
    digits = {c: O.modup(params, lv, cts[c].c1) for c in range(plan.col_blocks)}
    baby = {}
    outs = []
    for b in range(plan.row_blocks):
        out = None
        for c in range(plan.col_blocks):
            for j in range(g):
                acc0 = np.zeros((len(QPp), N), dtype=np.uint64)
                acc1 = np.zeros_like(acc0)
                for k in range(bs):
                    if (c, k) not in baby:
                        baby[(c, k)] = lazy_term(params, cts[c], digits[c], keys, k)
                    t0, t1 = baby[(c, k)]
                    i = j * bs + k
                    pt = O.reduce_signed(pt_ints[(b * plan.col_blocks + c) * plan.mprime + i], QPp)
                    for r, mod in enumerate(QPp):
                        acc0[r] = O.poly_add(acc0[r], O.poly_mul(pt[r], t0[r], mod), mod)
                        acc1[r] = O.poly_add(acc1[r], O.poly_mul(pt[r], t1[r], mod), mod)
                part = O.Ciphertext(O.moddown(params, lv, acc0), O.moddown(params, lv, acc1), lv)
                if j > 0:
                    gal = O.galois_rotl(j * bs, N)
                    part = O.hoisted_rotate(params, part, O.modup(params, lv, part.c1), keys[gal])
                out = part if out is None else O.ct_add(params, out, part)
        outs.append(out)
    return outs


def row_matmul(params: O.Params, plan: RowPlan, ct, pt_ints, ind_ints, keys: dict):
    """Sec. 3.1: per row r: pt_r*ct -> rescale -> log2 n x (t += RotL(t, 2^k))
    -> * indicator (encoded at scale q_{l-1}) -> rescale -> RotR(t, r); sum."""
    N = params.N
    lv = ct.level
    acc = None
    for r in range(plan.m):
        t = O.ct_mul_pt(params, ct, O.reduce_signed(pt_ints[r], params.q[: lv + 1]))
        t = O.rescale(params, t)
        for k in plan.ras_rotations():
            t = O.ct_add(params, t, O.rotate(params, t, keys[O.galois_rotl(k, N)]))
        t = O.ct_mul_pt(params, t, O.reduce_signed(ind_ints, params.q[: t.level + 1]))
        t = O.rescale(params, t)
        if r > 0:
            t = O.rotate(params, t, keys[O.galois_rotr(r, N)])
        acc = t if acc is None else O.ct_add(params, acc, t)
    return acc


def row_galois(plan: RowPlan, N: int) -> list:
    gs = [O.galois_rotl(k, N) for k in plan.ras_rotations()]
    gs += [O.galois_rotr(r, N) for r in range(1, plan.m)]
    return sorted(set(gs))


def diag_matmul(params: O.Params, plan: DiagPlan, ct, pt_ints, keys: dict, lazy: bool, hoisted: bool = True):
    """Eq. 5 with hoisted rotations (or, hoisted = False, O3 rotations as in
    GALA's diagonal method); optional in-ciphertext RaS with O3."""

    class _T:
        def terms(self_inner):
            return [(0, i, i, 0) for i in range(plan.ndiag)]

    out = hybrid_matmul(params, _T(), [ct], pt_ints, keys, lazy, hoisted)[0]
    for k in plan.ras_rotations():
        out = O.ct_add(params, out, O.rotate(params, out, keys[O.galois_rotl(k, params.N)]))
    return out


def diag_galois(plan: DiagPlan, N: int) -> list:
    gs = [O.galois_rotl(i, N) for i in range(1, plan.ndiag)]
    gs += [O.galois_rotl(k, N) for k in plan.ras_rotations()]
    return sorted(set(gs))


def ctmat_matmul(params: O.Params, plan: CtMatPlan, cts, pt_ints) -> list:
    """Alg. 3: out_k = sum_i [[e_i]] * w_{i,k}; no rotations, no key switching."""
    lv = cts[0].level
    outs = []
    for k in range(plan.n_out_cts):
        acc = O.zero_ct(params, lv)
        for i in range(plan.ndiag):
            pt = O.reduce_signed(pt_ints[i * plan.n_out_cts + k], params.q[: lv + 1])
            acc = O.ct_add(params, acc, O.ct_mul_pt(params, cts[i], pt))
        outs.append(acc)
    return outs


# ---------------------------------------------------------------------------
# Transposed diagonal conversion (Sec. 5.3, Eq. 7): the Eq. 5 diagonal
# ciphertexts of A^T from those of A, one rotation each.  As printed (RotR of
# diagonal (min - i) mod min by max - min + i) the equation does not
# reproduce A^T's diagonals for any tall shape; the reading below follows from
# e_k[j] = A[j mod m, (k + j) mod n] with the slots cyclic over max(m, n):
#   m >= n:  e'_i = RotL(e_((n - i) mod n), i)
#   m <  n:  e'_i = RotL(e_((m - i) mod m), n - m + i)  (i > 0),  e'_0 = e_0
# Rotating over all N' slots is cyclic over max(m, n) only when every block
# holds the diagonal, i.e. pack * max(m, n) = N'.
# ---------------------------------------------------------------------------
def transpose_map(plan: CtMatPlan) -> list:
    """(k, r) for every diagonal i of A^T: e'_i = RotL(e_k, r)"""
    lo, hi = plan.ndiag, plan.width
    out = []
    for i in range(lo):
        k = (lo - i) % lo
        if plan.mp >= plan.np_:
            r = i
        else:
            r = 0 if i == 0 else hi - lo + i
        out.append((k, r))
    return out


def transpose_map_as_printed(plan: CtMatPlan) -> list:
    """Eq. 7 read literally (RotR by max - min + i), for the pin that rejects it"""
    lo, hi = plan.ndiag, plan.width
    return [((lo - i) % lo, -((hi - lo + i) % hi)) for i in range(lo)]


def transpose_galois(plan: CtMatPlan, N: int) -> list:
    return sorted(set(O.galois_rotl(r, N) for _, r in transpose_map(plan) if r))


def ctmat_transpose(params: O.Params, plan: CtMatPlan, cts, keys: dict) -> list:
    """diagonal ciphertexts of A^T from those of A (unhoisted rotations, O3)"""
    assert plan.pack * plan.width == plan.slots, "the conversion needs every block to hold the diagonal"
    out = []
    for k, r in transpose_map(plan):
        out.append(cts[k] if r == 0 else O.rotate(params, cts[k], keys[O.galois_rotl(r, params.N)]))
    return out


# ---------------------------------------------------------------------------
# Sec. 5.2: multiplication-level reduction (Eq. 4), cleartext inverse RaS,
# and the masking of the result (Alg. 2)
# ---------------------------------------------------------------------------
def eq4_cleartext(q0: float, q1: float, q2: float, z, y, X):
    """The two sides of Eq. 4 in cleartext: CAESAR's gradient e^T X with
    e = q0 + q1 z + q2 z^3 - y, and its split (q0 1 - y)^T X + (q1 X)^T z +
    (q2 X)^T z^3.  X is batch x features."""
    e = q0 + q1 * z + q2 * z ** 3 - y
    lhs = e @ X
    rhs = (q0 * np.ones_like(y) - y) @ X + (q1 * X).T @ z + (q2 * X).T @ z ** 3
    return lhs, rhs


def inverse_ras(values, steps: int) -> np.ndarray:
    """Cleartext inverse RaS: `steps` rounds of splitting every value into two
    equal halves and concatenating the two copies, so [M0, M1] becomes
    [M0/2, M1/2, M0/2, M1/2] -- the paper's [M00, M10, M01, M11] with
    M_i = M_i0 + M_i1.  Halving is exact in binary64."""
    u = np.asarray(values, dtype=np.float64)
    for _ in range(steps):
        u = np.concatenate([u / 2, u / 2])
    return u


def _log2(x: int) -> int:
    return x.bit_length() - 1


def out_slots(plan, v, ras_in_ct: bool = False) -> list:
    """Slot vectors, one per output ciphertext, that carry the cleartext v
    (one value per output, CTMAT: the m x n_out matrix) through the plan's
    lazy RaS: the result of decrypting ct + encode(slots) and applying the
    lazy RaS is the product plus v."""
    S = plan.slots
    if isinstance(plan, HybridPlan):
        outs = []
        for b in range(plan.row_blocks):
            z = np.zeros(S)
            for g in range(plan.G):
                rows = [b * plan.bm + g * plan.mprime + r for r in range(plan.mprime)]
                vals = [v[r] if r < plan.m else 0.0 for r in rows]
                z[g * plan.bn:(g + 1) * plan.bn] = inverse_ras(vals, _log2(plan.bn // plan.mprime))
            outs.append(z)
        return outs
    if isinstance(plan, DiagPlan):
        z = np.zeros(S)
        if plan.mp >= plan.np_ or ras_in_ct or plan.ras == "rot":
            z[: plan.m] = v[: plan.m]
        else:
            vals = [v[r] if r < plan.m else 0.0 for r in range(plan.mp)]
            z[: plan.np_] = inverse_ras(vals, _log2(plan.np_ // plan.mp))
        return [z]
    if isinstance(plan, CtMatPlan):
        V = np.asarray(v).reshape(plan.m, plan.nout)
        outs = []
        for k in range(plan.n_out_cts):
            z = np.zeros(S)
            for blk in range(plan.pack):
                col = k * plan.pack + blk
                if col >= plan.nout:
                    continue
                if plan.mp >= plan.np_:
                    z[blk * plan.width: blk * plan.width + plan.m] = V[:, col]
                else:
                    vals = [V[r, col] if r < plan.m else 0.0 for r in range(plan.mp)]
                    z[blk * plan.width: blk * plan.width + plan.np_] = inverse_ras(vals, _log2(plan.np_ // plan.mp))
            outs.append(z)
        return outs
    raise ValueError("no cleartext term for this plan")


def encode_at_output(params: O.Params, slots_vec, lv: int, e: int) -> np.ndarray:
    """A cleartext as a plaintext at scale 2^e * Delta: encoded at Delta, its
    coefficient residues multiplied by 2^e mod q (Delta * 2^e is the output
    scale of a product without rescale).  Returns [lv+1][N] residues
    (coefficient domain)."""
    m = O.encode(slots_vec, params.N, params.scale)
    res = O.reduce_signed(m, params.q[: lv + 1])
    return np.stack([O.poly_scalar(res[i], pow(2, e, q), q) for i, q in enumerate(params.q[: lv + 1])])


def ct_add_plain(params: O.Params, ct, pt_res, sign: int):
    """O1 with a plaintext: (c0 + sign * pt, c1)."""
    lv = ct.level
    c0 = np.stack([(O.poly_add if sign > 0 else O.poly_sub)(ct.c0[i], pt_res[i], params.q[i]) for i in range(lv + 1)])
    return O.Ciphertext(c0, ct.c1.copy(), lv, ct.scale)


def hybrid_matmul_sum(params: O.Params, plan, terms: list, keys: dict) -> list:
    """Eq. 4 on the lazy plan: terms = [(cts, pt_ints)], every pair laid out
    by `plan`; all terms accumulate over Q u P and every output takes one
    ModDown."""
    N = params.N
    lv = terms[0][0][0].level
    QPp = params.qp(lv)
    tl = [(0, i, i, 0) for i in range(plan.ndiag)] if isinstance(plan, DiagPlan) else plan.terms()
    n_out = max(t[3] for t in tl) + 1
    acc0 = [np.zeros((len(QPp), N), dtype=np.uint64) for _ in range(n_out)]
    acc1 = [np.zeros((len(QPp), N), dtype=np.uint64) for _ in range(n_out)]
    for cts, pt_ints in terms:
        digits = {c: O.modup(params, lv, cts[c].c1) for c in set(t[0] for t in tl)}
        cache = {}
        for (c, i, k, b) in tl:
            if (c, i) not in cache:
                cache[(c, i)] = lazy_term(params, cts[c], digits[c], keys, i)
            t0, t1 = cache[(c, i)]
            pt = O.reduce_signed(pt_ints[k], QPp)
            for r, mod in enumerate(QPp):
                acc0[b][r] = O.poly_add(acc0[b][r], O.poly_mul(pt[r], t0[r], mod), mod)
                acc1[b][r] = O.poly_add(acc1[b][r], O.poly_mul(pt[r], t1[r], mod), mod)
    return [O.Ciphertext(O.moddown(params, lv, acc0[b]), O.moddown(params, lv, acc1[b]), lv)
            for b in range(n_out)]


def col_pt_ints(params: O.Params, plan: ColPlan, X, scale: float) -> list:
    """plaintext j * row_blocks + b: column j, row block b"""
    return [O.encode(col_pt_slots(plan, X, j, b), params.N, scale)
            for j in range(plan.n) for b in range(plan.row_blocks)]


def col_matmul(params: O.Params, plan: ColPlan, cts, pt_ints) -> list:
    """out_b = sum_j pt_{j,b} * ct_j (Sec. 3.1, column order)"""
    lv = cts[0].level
    Qp = params.q[: lv + 1]
    outs = []
    for b in range(plan.row_blocks):
        acc = O.zero_ct(params, lv)
        for j in range(plan.n):
            pt = O.reduce_signed(pt_ints[j * plan.row_blocks + b], Qp)
            acc = O.ct_add(params, acc, O.ct_mul_pt(params, cts[j], pt))
        outs.append(acc)
    return outs
