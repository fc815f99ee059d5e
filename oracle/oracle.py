"""Plain CPU oracle of the PackVFL packed-HE matrix product (arXiv 2405.00482).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP
library: the scalar arithmetic lives in ``ckks_oracle.c`` (``__int128`` and
``%``), the orchestration below follows the paper's steps in its notation.

Conventions (every one of them is part of the contract the GPU path must
meet bit for bit; the paper itself only says "Lattigo CKKS", Sec. 7):

* Ring Z_Q[X]/(X^N+1), N' = N/2 slots (Sec. 2.2).  RNS primes q_0..q_L for the
  ciphertext modulus and p_0..p_{alpha-1} for the key-switching modulus P.
  Digit j at level l holds q_{j*alpha} .. q_{min(j*alpha+alpha-1, l)};
  beta_l = ceil((l+1)/alpha).  Extended basis order: q_0..q_l, p_0..p_{alpha-1}.
* All polynomials here are in the COEFFICIENT domain, residues in [0, q).
* Randomness: Philox4x32-10 word ``rand64(seed, stream, index)`` (see the C
  file), streams:
      secret s           (0x01<<56)                          index = coefficient
      encryption a, limb i  (0x02<<56) | i
      encryption e       (0x03<<56)
      rotation key a_j, limb r (0x04<<56)|(j<<40)|(r<<24)|g   (r indexes Q_L u P)
      rotation key e_j   (0x05<<56)|(j<<40)|g
      public key a, limb i  (0x06<<56) | i;  public key e (0x07<<56)
      public-key encryption v (0x08<<56), e0 (0x09<<56), e1 (0x0A<<56)
  uniform mod q = floor(u q / 2^64); ternary = floor(3u / 2^64) - 1;
  error = CBD(21) = popcount(u & (2^21-1)) - popcount((u>>21) & (2^21-1)).
* Encode (canonical embedding, Cheon et al. 2017):
      m_k = round_half_away( 2*Delta/N * Re sum_{j<N'} z_j zeta^(-k*5^j) ),
  zeta = exp(i*pi/N); decode z_j = Re sum_k m_k zeta^(k*5^j) / Delta.
* RotL(x, i)[j] = x[j+i] (the paper's naive-method example, Sec. 3.1) is the
  automorphism X -> X^(5^i mod 2N).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

U64P = ctypes.POINTER(ctypes.c_uint64)
I64P = ctypes.POINTER(ctypes.c_int64)
U32P = ctypes.POINTER(ctypes.c_uint32)


def build_oracle(force: bool = False) -> str:
    """Compile the C core with gcc (plain -O2, no vector intrinsics)."""
    src = os.path.join(_HERE, "ckks_oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        import subprocess
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build_oracle()
        L = ctypes.CDLL(_LIB_PATH)
        u64 = ctypes.c_uint64
        L.or_mulmod.restype = u64
        L.or_mulmod.argtypes = [u64, u64, u64]
        L.or_powmod.restype = u64
        L.or_powmod.argtypes = [u64, u64, u64]
        L.or_invmod.restype = u64
        L.or_invmod.argtypes = [u64, u64]
        L.or_is_prime.restype = ctypes.c_int
        L.or_is_prime.argtypes = [u64]
        L.or_psi.restype = u64
        L.or_psi.argtypes = [u64, ctypes.c_int]
        L.or_rand64.restype = u64
        L.or_rand64.argtypes = [u64, u64, u64]
        L.or_philox4x32_10.restype = None
        L.or_philox4x32_10.argtypes = [U32P, U32P, U32P]
        L.or_sample_uniform.argtypes = [u64, u64, u64, ctypes.c_int, U64P]
        L.or_sample_ternary.argtypes = [u64, u64, ctypes.c_int, I64P]
        L.or_sample_cbd21.argtypes = [u64, u64, ctypes.c_int, I64P]
        L.or_ntt_forward.argtypes = [U64P, ctypes.c_int, u64, u64]
        L.or_ntt_inverse.argtypes = [U64P, ctypes.c_int, u64, u64]
        L.or_negacyclic_mul.argtypes = [U64P, U64P, U64P, ctypes.c_int, u64]
        L.or_negacyclic_mul_schoolbook.argtypes = [U64P, U64P, U64P, ctypes.c_int, u64]
        for nm in ("or_poly_add", "or_poly_sub"):
            getattr(L, nm).argtypes = [U64P, U64P, U64P, ctypes.c_int, u64]
        L.or_poly_neg.argtypes = [U64P, U64P, ctypes.c_int, u64]
        L.or_poly_scalar_mul.argtypes = [U64P, u64, U64P, ctypes.c_int, u64]
        L.or_poly_from_signed.argtypes = [I64P, U64P, ctypes.c_int, u64]
        L.or_automorphism.argtypes = [U64P, U64P, ctypes.c_int, u64, u64]
        L.or_base_convert.argtypes = [U64P, U64P, ctypes.c_int, u64, U64P, ctypes.c_int]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    if a.dtype == np.uint64:
        return a.ctypes.data_as(U64P)
    if a.dtype == np.int64:
        return a.ctypes.data_as(I64P)
    if a.dtype == np.uint32:
        return a.ctypes.data_as(U32P)
    raise TypeError(a.dtype)


# ---------------------------------------------------------------------------
# scalar helpers
# ---------------------------------------------------------------------------
def mulmod(a: int, b: int, q: int) -> int:
    return (a * b) % q


def invmod(a: int, q: int) -> int:
    return pow(a % q, q - 2, q)


def is_prime(n: int) -> bool:
    return bool(lib().or_is_prime(n))


def philox4x32_10(ctr, key):
    c = np.array(ctr, dtype=np.uint32)
    k = np.array(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(o))
    return [int(x) for x in o]


def rand64(seed: int, stream: int, idx: int) -> int:
    return int(lib().or_rand64(seed, stream, idx))


# streams
def stream_secret() -> int:
    return 0x01 << 56


def stream_enc_a(limb: int) -> int:
    return (0x02 << 56) | limb


def stream_enc_e() -> int:
    return 0x03 << 56


def stream_key_a(j: int, r: int, g: int) -> int:
    return (0x04 << 56) | (j << 40) | (r << 24) | g


def stream_key_e(j: int, g: int) -> int:
    return (0x05 << 56) | (j << 40) | g


def stream_pk_a(limb: int) -> int:
    return (0x06 << 56) | limb


def stream_pk_e() -> int:
    return 0x07 << 56


def stream_pkenc(part: str) -> int:
    return {"v": 0x08, "e0": 0x09, "e1": 0x0A}[part] << 56


def sample_uniform(seed, stream, q, n) -> np.ndarray:
    out = np.zeros(n, dtype=np.uint64)
    lib().or_sample_uniform(seed, stream, q, n, _p(out))
    return out


def sample_ternary(seed, stream, n) -> np.ndarray:
    out = np.zeros(n, dtype=np.int64)
    lib().or_sample_ternary(seed, stream, n, _p(out))
    return out


def sample_cbd21(seed, stream, n) -> np.ndarray:
    out = np.zeros(n, dtype=np.int64)
    lib().or_sample_cbd21(seed, stream, n, _p(out))
    return out


# ---------------------------------------------------------------------------
# single-limb polynomial operations (coefficient domain)
# ---------------------------------------------------------------------------
def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint64)


def poly_mul(a, b, q) -> np.ndarray:
    a, b = _c(a), _c(b)
    out = np.zeros_like(a)
    lib().or_negacyclic_mul(_p(a), _p(b), _p(out), a.size, q)
    return out


def poly_mul_schoolbook(a, b, q) -> np.ndarray:
    a, b = _c(a), _c(b)
    out = np.zeros_like(a)
    lib().or_negacyclic_mul_schoolbook(_p(a), _p(b), _p(out), a.size, q)
    return out


def poly_add(a, b, q) -> np.ndarray:
    a, b = _c(a), _c(b)
    out = np.zeros_like(a)
    lib().or_poly_add(_p(a), _p(b), _p(out), a.size, q)
    return out


def poly_sub(a, b, q) -> np.ndarray:
    a, b = _c(a), _c(b)
    out = np.zeros_like(a)
    lib().or_poly_sub(_p(a), _p(b), _p(out), a.size, q)
    return out


def poly_neg(a, q) -> np.ndarray:
    a = _c(a)
    out = np.zeros_like(a)
    lib().or_poly_neg(_p(a), _p(out), a.size, q)
    return out


def poly_scalar(a, c, q) -> np.ndarray:
    a = _c(a)
    out = np.zeros_like(a)
    lib().or_poly_scalar_mul(_p(a), c % q, _p(out), a.size, q)
    return out


def poly_from_signed(a, q) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.int64)
    out = np.zeros(a.size, dtype=np.uint64)
    lib().or_poly_from_signed(_p(a), _p(out), a.size, q)
    return out


def poly_from_ints(vals, q) -> np.ndarray:
    """Reduce arbitrary Python integers into [0, q)."""
    return np.array([int(v) % q for v in vals], dtype=np.uint64)


def automorphism(a, g, q) -> np.ndarray:
    a = _c(a)
    out = np.zeros_like(a)
    lib().or_automorphism(_p(a), _p(out), a.size, q, g)
    return out


def ntt_forward(a, q) -> np.ndarray:
    """The oracle's own negacyclic NTT (natural order of exponents 2k+1)."""
    a = _c(a).copy()
    lib().or_ntt_forward(_p(a), a.size, q, lib().or_psi(q, a.size))
    return a


def ntt_inverse(a, q) -> np.ndarray:
    a = _c(a).copy()
    lib().or_ntt_inverse(_p(a), a.size, q, lib().or_psi(q, a.size))
    return a


def psi(q: int, N: int) -> int:
    return int(lib().or_psi(q, N))


def base_convert(limbs, B, r) -> np.ndarray:
    """Conv_{B->r} of len(B) coefficient limbs (fast base conversion)."""
    x = np.ascontiguousarray(np.stack([_c(l) for l in limbs]), dtype=np.uint64)
    Barr = np.ascontiguousarray(B, dtype=np.uint64)
    N = x.shape[1]
    out = np.zeros(N, dtype=np.uint64)
    lib().or_base_convert(_p(x), _p(Barr), len(B), r, _p(out), N)
    return out


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------
@dataclass
class Params:
    logN: int
    q: list          # ciphertext primes q_0..q_L
    p: list          # special primes p_0..p_{alpha-1}
    log2_scale: float
    name: str = ""

    @property
    def N(self) -> int:
        return 1 << self.logN

    @property
    def slots(self) -> int:
        return self.N // 2

    @property
    def L(self) -> int:
        return len(self.q) - 1

    @property
    def alpha(self) -> int:
        return len(self.p)

    @property
    def scale(self) -> float:
        return 2.0 ** self.log2_scale

    def beta(self, level: int) -> int:
        return -(-(level + 1) // self.alpha)

    def digit(self, level: int, j: int) -> list:
        """indices (into q) of the primes of digit j at this level"""
        lo = j * self.alpha
        hi = min(lo + self.alpha - 1, level)
        return list(range(lo, hi + 1))

    def qp(self, level: int) -> list:
        """extended basis Q_l u P, in storage order"""
        return list(self.q[: level + 1]) + list(self.p)

    def P(self) -> int:
        return math.prod(self.p)

    def Q(self, level: int) -> int:
        return math.prod(self.q[: level + 1])

    @staticmethod
    def from_dict(d: dict) -> "Params":
        return Params(logN=int(d["logN"]), q=[int(x) for x in d["q"]], p=[int(x) for x in d["p"]],
                      log2_scale=float(d["log2_scale"]), name=d.get("name", ""))


def galois_rotl(i: int, N: int) -> int:
    """Galois element of RotL by i slots: 5^i mod 2N (5 has order N/2)."""
    return pow(5, i % (N // 2), 2 * N)


def galois_rotr(i: int, N: int) -> int:
    return pow(5, (N // 2 - (i % (N // 2))) % (N // 2), 2 * N)


# ---------------------------------------------------------------------------
# encoding (canonical embedding)
# ---------------------------------------------------------------------------
def _slot_exponents(N: int) -> np.ndarray:
    e = np.empty(N // 2, dtype=np.int64)
    x = 1
    for j in range(N // 2):
        e[j] = x
        x = (x * 5) % (2 * N)
    return e


def round_half_away(x: np.ndarray) -> np.ndarray:
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def encode(z, N: int, scale: float) -> np.ndarray:
    """Real slot vector (length <= N/2, zero-filled) -> int64 coefficients.

    m_k = (scale/N) * FFT_2N(w)[k] with w[5^j] = z_j and w[-5^j] = conj(z_j),
    which is the inverse canonical embedding written as one length-2N DFT.
    """
    z = np.asarray(z, dtype=np.complex128)
    zz = np.zeros(N // 2, dtype=np.complex128)
    zz[: z.size] = z
    e = _slot_exponents(N)
    w = np.zeros(2 * N, dtype=np.complex128)
    w[e] = zz
    w[(2 * N - e) % (2 * N)] = np.conj(zz)
    F = np.fft.fft(w)
    v = (scale / N) * F[:N].real
    return round_half_away(v).astype(np.int64)


def encode_direct(z, N: int, scale: float) -> np.ndarray:
    """O(N^2) direct sum of the encoding formula (tiny N pins)."""
    z = np.asarray(z, dtype=np.float64)
    e = _slot_exponents(N)
    out = np.zeros(N, dtype=np.float64)
    for k in range(N):
        s = 0.0
        for j in range(z.size):
            s += z[j] * math.cos(-math.pi * k * int(e[j]) / N)
        out[k] = 2.0 * scale / N * s
    return round_half_away(out).astype(np.int64)


def decode(m_ints, N: int, scale: float) -> np.ndarray:
    """Integer coefficients (Python ints, any size) -> real slots."""
    mf = np.array([float(int(v)) for v in m_ints], dtype=np.float64)
    v = np.fft.ifft(np.concatenate([mf, np.zeros(N)])) * (2 * N)
    e = _slot_exponents(N)
    return v[e].real / scale


# ---------------------------------------------------------------------------
# multi-limb helpers
# ---------------------------------------------------------------------------
def reduce_signed(m, primes) -> np.ndarray:
    """int64 (or Python int) coefficient vector -> [len(primes)][N] residues."""
    m = np.asarray(m)
    if m.dtype == np.int64:
        return np.stack([poly_from_signed(m, q) for q in primes])
    return np.stack([poly_from_ints(m, q) for q in primes])


def crt_centered(res, primes) -> list:
    """Residues [k][N] -> centred integers in (-Q/2, Q/2] (Python ints)."""
    Q = math.prod(primes)
    N = res.shape[1]
    coef = []
    for i, q in enumerate(primes):
        Qi = Q // q
        coef.append((Qi * invmod(Qi % q, q)) % Q)
    out = []
    for k in range(N):
        x = 0
        for i in range(len(primes)):
            x += int(res[i, k]) * coef[i]
        x %= Q
        if x > Q // 2:
            x -= Q
        out.append(x)
    return out


# ---------------------------------------------------------------------------
# keys and encryption (Sec. 2.2)
# ---------------------------------------------------------------------------
def keygen(params: Params, seed: int) -> np.ndarray:
    """Ternary secret s as int64[N]."""
    return sample_ternary(seed, stream_secret(), params.N)


def _limbs_of(params: Params, ints, primes):
    return reduce_signed(ints, primes)


@dataclass
class Ciphertext:
    c0: np.ndarray      # [l+1][N] uint64, coefficient domain
    c1: np.ndarray
    level: int
    scale: float = 1.0

    def copy(self):
        return Ciphertext(self.c0.copy(), self.c1.copy(), self.level, self.scale)


def encrypt(params: Params, s, m, level: int, seed: int, scale: float = 1.0) -> Ciphertext:
    """Secret-key RLWE encryption (Sec. 2.2): c1 = a, c0 = -a*s + m + e."""
    N = params.N
    primes = params.q[: level + 1]
    e = sample_cbd21(seed, stream_enc_e(), N)
    mres = reduce_signed(m, primes)
    c0 = np.zeros((level + 1, N), dtype=np.uint64)
    c1 = np.zeros((level + 1, N), dtype=np.uint64)
    for i, q in enumerate(primes):
        a = sample_uniform(seed, stream_enc_a(i), q, N)
        s_q = poly_from_signed(s, q)
        as_ = poly_mul(a, s_q, q)
        c0[i] = poly_add(poly_sub(mres[i], as_, q), poly_from_signed(e, q), q)
        c1[i] = a
    return Ciphertext(c0, c1, level, scale)


def pk_gen(params: Params, s, seed: int):
    """Public key (b, a) = (-a s + e, a) over the L+1 ciphertext primes
    (coefficient domain): the public-key form of RLWE encryption."""
    N = params.N
    e = sample_cbd21(seed, stream_pk_e(), N)
    b, a = [], []
    for i, q in enumerate(params.q):
        ai = sample_uniform(seed, stream_pk_a(i), q, N)
        b.append(poly_add(poly_sub(np.zeros(N, dtype=np.uint64), poly_mul(ai, poly_from_signed(s, q), q), q),
                          poly_from_signed(e, q), q))
        a.append(ai)
    return np.stack(b), np.stack(a)


def encrypt_pk(params: Params, pk, m, level: int, seed: int, scale: float = 1.0) -> Ciphertext:
    """Public-key encryption: v ternary, c0 = v b + m + e0, c1 = v a + e1."""
    N = params.N
    b, a = pk
    v = sample_ternary(seed, stream_pkenc("v"), N)
    e0 = sample_cbd21(seed, stream_pkenc("e0"), N)
    e1 = sample_cbd21(seed, stream_pkenc("e1"), N)
    primes = params.q[: level + 1]
    mres = reduce_signed(m, primes)
    c0 = np.zeros((level + 1, N), dtype=np.uint64)
    c1 = np.zeros((level + 1, N), dtype=np.uint64)
    for i, q in enumerate(primes):
        vq = poly_from_signed(v, q)
        c0[i] = poly_add(poly_add(poly_mul(vq, b[i], q), mres[i], q), poly_from_signed(e0, q), q)
        c1[i] = poly_add(poly_mul(vq, a[i], q), poly_from_signed(e1, q), q)
    return Ciphertext(c0, c1, level, scale)


def decrypt(params: Params, s, ct: Ciphertext) -> np.ndarray:
    """c0 + c1*s per limb; residues [l+1][N]."""
    out = np.zeros_like(ct.c0)
    for i, q in enumerate(params.q[: ct.level + 1]):
        out[i] = poly_add(ct.c0[i], poly_mul(ct.c1[i], poly_from_signed(s, q), q), q)
    return out


def decrypt_decode(params: Params, s, ct: Ciphertext, scale: float) -> np.ndarray:
    res = decrypt(params, s, ct)
    m = crt_centered(res, params.q[: ct.level + 1])
    return decode(m, params.N, scale)


@dataclass
class SwitchKey:
    """b_j, a_j for j < beta_L over Q_L u P (coefficient domain)."""
    g: int
    b: list   # [beta_L] of [L+1+alpha][N]
    a: list


def rotkey_gen(params: Params, s, g: int, seed: int) -> SwitchKey:
    """Key switching from s' = phi_g(s) to s (hybrid key switching, Han-Ki 2020):
        b_j = -a_j*s + e_j + [r in D_j] * (P mod r) * s'   (mod every r in Q_L u P)
    """
    N = params.N
    L = params.L
    basis = params.qp(L)
    Pint = params.P()
    bL = params.beta(L)
    bs, as_ = [], []
    for j in range(bL):
        digit = params.digit(L, j)
        e = sample_cbd21(seed, stream_key_e(j, g), N)
        bj = np.zeros((len(basis), N), dtype=np.uint64)
        aj = np.zeros((len(basis), N), dtype=np.uint64)
        for r, mod in enumerate(basis):
            a = sample_uniform(seed, stream_key_a(j, r, g), mod, N)
            s_r = poly_from_signed(s, mod)
            b = poly_add(poly_neg(poly_mul(a, s_r, mod), mod), poly_from_signed(e, mod), mod)
            if r <= L and r in digit:
                sp = automorphism(s_r, g, mod)
                b = poly_add(b, poly_scalar(sp, Pint % mod, mod), mod)
            bj[r] = b
            aj[r] = a
        bs.append(bj)
        as_.append(aj)
    return SwitchKey(g, bs, as_)


def key_at_level(params: Params, key: SwitchKey, level: int):
    """Restrict a level-L key to Q_level u P and beta_level digits."""
    L = params.L
    idx = list(range(level + 1)) + list(range(L + 1, L + 1 + params.alpha))
    bl = params.beta(level)
    return [key.b[j][idx] for j in range(bl)], [key.a[j][idx] for j in range(bl)]


# ---------------------------------------------------------------------------
# ModUp / ModDown / Rescale (full-RNS CKKS, Cheon et al. SAC 2018)
# ---------------------------------------------------------------------------
def modup(params: Params, level: int, d) -> list:
    """Digits D_j of d (coefficient domain, [l+1][N]) over Q_l u P.

    Residues of digit j are kept; every other limb gets Conv_{D_j -> r}.
    """
    basis = params.qp(level)
    out = []
    for j in range(params.beta(level)):
        dig = params.digit(level, j)
        Dj = np.zeros((len(basis), params.N), dtype=np.uint64)
        src = [d[i] for i in dig]
        Bj = [params.q[i] for i in dig]
        for r, mod in enumerate(basis):
            if r <= level and r in dig:
                Dj[r] = d[r]
            else:
                Dj[r] = base_convert(src, Bj, mod)
        out.append(Dj)
    return out


def moddown(params: Params, level: int, u) -> np.ndarray:
    """Q_l u P -> Q_l with rounding, coefficient-wise: add floor(P/2) to every
    coefficient, subtract Conv_{P->q_i} of the P part, multiply by P^-1 mod q_i.
    Result: round(u/P) - w with 0 <= w < alpha (the conversion's overshoot)."""
    N = params.N
    P = params.P()
    h = P // 2
    basis = params.qp(level)
    up = []
    for r, mod in enumerate(basis):
        # round(u/P) coefficient-wise: floor-division of u + floor(P/2)
        up.append(poly_add(u[r], np.full(N, h % mod, dtype=np.uint64), mod))
    uP = up[level + 1:]
    out = np.zeros((level + 1, N), dtype=np.uint64)
    for i in range(level + 1):
        q = params.q[i]
        t = base_convert(uP, params.p, q)
        out[i] = poly_scalar(poly_sub(up[i], t, q), invmod(P % q, q), q)
    return out


def rescale_poly(params: Params, level: int, c) -> np.ndarray:
    """Drop q_level with rounding: the ModDown formula with P := q_level."""
    ql = params.q[level]
    h = ql // 2
    N = params.N
    x = [poly_add(c[i], np.full(N, h % params.q[i], dtype=np.uint64), params.q[i]) for i in range(level + 1)]
    out = np.zeros((level, params.N), dtype=np.uint64)
    for i in range(level):
        q = params.q[i]
        t = base_convert([x[level]], [ql], q)
        out[i] = poly_scalar(poly_sub(x[i], t, q), invmod(ql % q, q), q)
    return out


def rescale(params: Params, ct: Ciphertext) -> Ciphertext:
    ql = params.q[ct.level]
    return Ciphertext(rescale_poly(params, ct.level, ct.c0), rescale_poly(params, ct.level, ct.c1),
                      ct.level - 1, ct.scale / ql)


# ---------------------------------------------------------------------------
# key switching and rotations (O3, O4 of Sec. 2.2)
# ---------------------------------------------------------------------------
def inner_product(params: Params, level: int, digits, key: SwitchKey, g_apply: int | None):
    """(u0, u1) = sum_j phi_g(D_j) * (b_j, a_j) over Q_l u P.

    g_apply: automorphism applied to every extended digit first (hoisting);
    None when the digits were taken of an already-rotated polynomial.
    """
    basis = params.qp(level)
    kb, ka = key_at_level(params, key, level)
    u0 = np.zeros((len(basis), params.N), dtype=np.uint64)
    u1 = np.zeros_like(u0)
    for j, Dj in enumerate(digits):
        for r, mod in enumerate(basis):
            d = Dj[r] if g_apply is None else automorphism(Dj[r], g_apply, mod)
            u0[r] = poly_add(u0[r], poly_mul(d, kb[j][r], mod), mod)
            u1[r] = poly_add(u1[r], poly_mul(d, ka[j][r], mod), mod)
    return u0, u1


def automorphism_ct_part(params: Params, level: int, c, g):
    return np.stack([automorphism(c[i], g, params.q[i]) for i in range(level + 1)])


def rotate(params: Params, ct: Ciphertext, key: SwitchKey) -> Ciphertext:
    """O3: unhoisted rotation.  (phi_g c0 + ModDown(u0), ModDown(u1)) with
    (u0, u1) = KS(phi_g c1): the automorphism precedes ModUp."""
    lv = ct.level
    g = key.g
    c0r = automorphism_ct_part(params, lv, ct.c0, g)
    c1r = automorphism_ct_part(params, lv, ct.c1, g)
    digits = modup(params, lv, c1r)
    u0, u1 = inner_product(params, lv, digits, key, None)
    v0 = moddown(params, lv, u0)
    v1 = moddown(params, lv, u1)
    c0 = np.stack([poly_add(c0r[i], v0[i], params.q[i]) for i in range(lv + 1)])
    return Ciphertext(c0, v1, lv, ct.scale)


def hoisted_rotate(params: Params, ct: Ciphertext, digits, key: SwitchKey) -> Ciphertext:
    """O4: hoisted rotation; digits = modup(c1) computed once per ciphertext and
    the automorphism applied to the extended digits (ModUp precedes phi_g)."""
    lv = ct.level
    g = key.g
    u0, u1 = inner_product(params, lv, digits, key, g)
    v0 = moddown(params, lv, u0)
    v1 = moddown(params, lv, u1)
    c0r = automorphism_ct_part(params, lv, ct.c0, g)
    c0 = np.stack([poly_add(c0r[i], v0[i], params.q[i]) for i in range(lv + 1)])
    return Ciphertext(c0, v1, lv, ct.scale)


# ---------------------------------------------------------------------------
# ciphertext-plaintext products (O1, O2)
# ---------------------------------------------------------------------------
def ct_add(params: Params, a: Ciphertext, b: Ciphertext) -> Ciphertext:
    assert a.level == b.level
    c0 = np.stack([poly_add(a.c0[i], b.c0[i], params.q[i]) for i in range(a.level + 1)])
    c1 = np.stack([poly_add(a.c1[i], b.c1[i], params.q[i]) for i in range(a.level + 1)])
    return Ciphertext(c0, c1, a.level, a.scale)


def ct_mul_pt(params: Params, ct: Ciphertext, pt_res, pt_scale: float = 1.0) -> Ciphertext:
    """pt_res: [>= l+1][N] residues of the plaintext polynomial."""
    lv = ct.level
    c0 = np.stack([poly_mul(ct.c0[i], pt_res[i], params.q[i]) for i in range(lv + 1)])
    c1 = np.stack([poly_mul(ct.c1[i], pt_res[i], params.q[i]) for i in range(lv + 1)])
    return Ciphertext(c0, c1, lv, ct.scale * pt_scale)


def zero_ct(params: Params, level: int, scale: float = 1.0) -> Ciphertext:
    z = np.zeros((level + 1, params.N), dtype=np.uint64)
    return Ciphertext(z, z.copy(), level, scale)
