/*
 * Plain CPU oracle for the packed-HE (RNS-CKKS) ciphertext x plaintext matrix
 * product of PackVFL (arXiv 2405.00482).  TEST INFRASTRUCTURE ONLY: nothing in
 * the product path may link, load or call this file; only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark do.
 *
 * Everything here is scalar, single-threaded C over unsigned 64-bit residues
 * with unsigned __int128 products and the % operator.  Polynomials live in the
 * coefficient domain of Z_q[X]/(X^N+1); the NTT below is used only as the means
 * of computing a negacyclic product, never as a storage format, so its choice
 * of root and ordering is invisible to callers.
 *
 * Sources of the mathematics (the paper only names "Lattigo CKKS", Sec. 7):
 *   - RLWE encryption/decryption: Sec. 2.2 (Packed Homomorphic Encryption).
 *   - full-RNS CKKS base conversion: Cheon-Han-Kim-Kim-Song, SAC 2018, and
 *     Bajard-Eynard-Hasan-Zucca, SAC 2016 (fast base extension, no overflow
 *     correction).
 *   - negacyclic NTT: the textbook "twist by psi^j, then cyclic DFT by
 *     omega = psi^2" construction.
 *   - Philox4x32-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 *     as easy as 1, 2, 3", SC'11.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* scalar modular arithmetic (q < 2^62)                                 */
/* ------------------------------------------------------------------ */
u64 or_mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * (u128)b) % q); }
static u64 addmod(u64 a, u64 b, u64 q) { u64 s = (a % q) + (b % q); return s >= q ? s - q : s; }
static u64 submod(u64 a, u64 b, u64 q) { a %= q; b %= q; return a >= b ? a - b : a + q - b; }

u64 or_powmod(u64 a, u64 e, u64 q) {
  u64 r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = or_mulmod(r, a, q);
    a = or_mulmod(a, a, q);
    e >>= 1;
  }
  return r;
}

/* inverse modulo a prime q, by Fermat's little theorem */
u64 or_invmod(u64 a, u64 q) { return or_powmod(a, q - 2, q); }

/* deterministic Miller-Rabin, valid for all n < 3.3e24 with these bases */
int or_is_prime(u64 n) {
  static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; ++i) {
    if (n == bases[i]) return 1;
    if (n % bases[i] == 0) return 0;
  }
  u64 d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (int i = 0; i < 12; ++i) {
    u64 x = or_powmod(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int comp = 1;
    for (int r = 1; r < s; ++r) {
      x = or_mulmod(x, x, n);
      if (x == n - 1) { comp = 0; break; }
    }
    if (comp) return 0;
  }
  return 1;
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11)                                 */
/* ------------------------------------------------------------------ */
static void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  u64 p = (u64)a * (u64)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

/* ctr[4], key[2] in; out[4] */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += W0; k1 += W1; }
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo32(M0, c0, &hi0, &lo0);
    mulhilo32(M1, c2, &hi1, &lo1);
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/*
 * The library-wide counter-based generator: word number `idx` of stream
 * `stream` under key `seed`.  Philox counter = (idx>>1 as two 32-bit words,
 * stream as two 32-bit words), key = seed as two 32-bit words; the even index
 * takes output words (0,1), the odd index words (2,3), low word first.
 */
u64 or_rand64(u64 seed, u64 stream, u64 idx) {
  uint32_t ctr[4], key[2], out[4];
  u64 blk = idx >> 1;
  ctr[0] = (uint32_t)blk; ctr[1] = (uint32_t)(blk >> 32);
  ctr[2] = (uint32_t)stream; ctr[3] = (uint32_t)(stream >> 32);
  key[0] = (uint32_t)seed; key[1] = (uint32_t)(seed >> 32);
  or_philox4x32_10(ctr, key, out);
  if (idx & 1) return (u64)out[2] | ((u64)out[3] << 32);
  return (u64)out[0] | ((u64)out[1] << 32);
}

/* uniform residue in [0, q): floor(u * q / 2^64) */
void or_sample_uniform(u64 seed, u64 stream, u64 q, int n, u64* out) {
  for (int k = 0; k < n; ++k) {
    u64 u = or_rand64(seed, stream, (u64)k);
    out[k] = (u64)(((u128)u * (u128)q) >> 64);
  }
}

/* uniform ternary in {-1, 0, 1}: floor(u * 3 / 2^64) - 1 */
void or_sample_ternary(u64 seed, u64 stream, int n, int64_t* out) {
  for (int k = 0; k < n; ++k) {
    u64 u = or_rand64(seed, stream, (u64)k);
    out[k] = (int64_t)(((u128)u * 3u) >> 64) - 1;
  }
}

static int popcount64(u64 x) {
  int c = 0;
  while (x) { x &= x - 1; ++c; }
  return c;
}

/* centred binomial with eta = 21: popcount of 21 bits minus popcount of the next 21 */
void or_sample_cbd21(u64 seed, u64 stream, int n, int64_t* out) {
  const u64 mask = (1ull << 21) - 1;
  for (int k = 0; k < n; ++k) {
    u64 u = or_rand64(seed, stream, (u64)k);
    out[k] = (int64_t)popcount64(u & mask) - (int64_t)popcount64((u >> 21) & mask);
  }
}

/* ------------------------------------------------------------------ */
/* roots of unity                                                      */
/* ------------------------------------------------------------------ */
/* smallest quadratic non-residue modulo the odd prime q (Euler's criterion) */
u64 or_smallest_nonresidue(u64 q) {
  for (u64 x = 2;; ++x)
    if (or_powmod(x, (q - 1) / 2, q) == q - 1) return x;
}

/* primitive 2N-th root of unity: nu^((q-1)/2N) with nu a non-residue, so psi^N = -1 */
u64 or_psi(u64 q, int N) {
  if ((q - 1) % (2 * (u64)N) != 0) abort(); /* q must be 1 mod 2N */
  u64 nu = or_smallest_nonresidue(q);
  return or_powmod(nu, (q - 1) / (2 * (u64)N), q);
}

/* ------------------------------------------------------------------ */
/* negacyclic NTT: A[k] = sum_j a_j psi^((2k+1) j), k in natural order  */
/* ------------------------------------------------------------------ */
static void bit_reverse_permute(u64* a, int n) {
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) { u64 t = a[i]; a[i] = a[j]; a[j] = t; }
  }
}

/* in-place cyclic DFT of length n over Z_q with primitive n-th root w */
static void cyclic_dft(u64* a, int n, u64 w, u64 q) {
  bit_reverse_permute(a, n);
  for (int len = 2; len <= n; len <<= 1) {
    u64 wl = or_powmod(w, (u64)(n / len), q);
    for (int i = 0; i < n; i += len) {
      u64 x = 1;
      for (int j = 0; j < len / 2; ++j) {
        u64 u = a[i + j];
        u64 v = or_mulmod(a[i + j + len / 2], x, q);
        a[i + j] = addmod(u, v, q);
        a[i + j + len / 2] = submod(u, v, q);
        x = or_mulmod(x, wl, q);
      }
    }
  }
}

/* forward: twist by psi^j, then cyclic DFT with omega = psi^2 */
void or_ntt_forward(u64* a, int N, u64 q, u64 psi) {
  u64 t = 1;
  for (int j = 0; j < N; ++j) { a[j] = or_mulmod(a[j] % q, t, q); t = or_mulmod(t, psi, q); }
  cyclic_dft(a, N, or_mulmod(psi, psi, q), q);
}

/* inverse: inverse cyclic DFT, scale by N^-1, untwist by psi^-j */
void or_ntt_inverse(u64* a, int N, u64 q, u64 psi) {
  u64 psi_inv = or_invmod(psi, q);
  cyclic_dft(a, N, or_mulmod(psi_inv, psi_inv, q), q);
  u64 n_inv = or_invmod((u64)N % q, q);
  u64 t = n_inv;
  for (int j = 0; j < N; ++j) { a[j] = or_mulmod(a[j], t, q); t = or_mulmod(t, psi_inv, q); }
}

/* out = a * b in Z_q[X]/(X^N + 1); out may alias a or b */
void or_negacyclic_mul(const u64* a, const u64* b, u64* out, int N, u64 q) {
  u64 psi = or_psi(q, N);
  u64* fa = (u64*)malloc(sizeof(u64) * (size_t)N);
  u64* fb = (u64*)malloc(sizeof(u64) * (size_t)N);
  for (int j = 0; j < N; ++j) { fa[j] = a[j] % q; fb[j] = b[j] % q; }
  or_ntt_forward(fa, N, q, psi);
  or_ntt_forward(fb, N, q, psi);
  for (int j = 0; j < N; ++j) fa[j] = or_mulmod(fa[j], fb[j], q);
  or_ntt_inverse(fa, N, q, psi);
  memcpy(out, fa, sizeof(u64) * (size_t)N);
  free(fa);
  free(fb);
}

/* schoolbook negacyclic product, O(N^2): the definition, for pinning the NTT */
void or_negacyclic_mul_schoolbook(const u64* a, const u64* b, u64* out, int N, u64 q) {
  u64* acc = (u64*)calloc((size_t)N, sizeof(u64));
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      u64 p = or_mulmod(a[i] % q, b[j] % q, q);
      int k = i + j;
      if (k < N) acc[k] = addmod(acc[k], p, q);
      else acc[k - N] = submod(acc[k - N], p, q); /* X^N = -1 */
    }
  memcpy(out, acc, sizeof(u64) * (size_t)N);
  free(acc);
}

/* ------------------------------------------------------------------ */
/* element-wise helpers on one limb                                    */
/* ------------------------------------------------------------------ */
void or_poly_add(const u64* a, const u64* b, u64* out, int N, u64 q) {
  for (int j = 0; j < N; ++j) out[j] = addmod(a[j], b[j], q);
}
void or_poly_sub(const u64* a, const u64* b, u64* out, int N, u64 q) {
  for (int j = 0; j < N; ++j) out[j] = submod(a[j], b[j], q);
}
void or_poly_neg(const u64* a, u64* out, int N, u64 q) {
  for (int j = 0; j < N; ++j) out[j] = submod(0, a[j], q);
}
void or_poly_scalar_mul(const u64* a, u64 c, u64* out, int N, u64 q) {
  for (int j = 0; j < N; ++j) out[j] = or_mulmod(a[j] % q, c % q, q);
}
/* reduce signed integer coefficients into [0, q) */
void or_poly_from_signed(const int64_t* a, u64* out, int N, u64 q) {
  for (int j = 0; j < N; ++j) {
    int64_t v = a[j] % (int64_t)q;
    if (v < 0) v += (int64_t)q;
    out[j] = (u64)v;
  }
}

/*
 * Galois automorphism phi_g: X -> X^g (g odd) in the coefficient domain.
 * Coefficient j moves to j*g mod 2N, negated when that exponent is >= N
 * (because X^N = -1).
 */
void or_automorphism(const u64* a, u64* out, int N, u64 q, u64 g) {
  u64 two_n = 2 * (u64)N;
  for (int j = 0; j < N; ++j) {
    u64 e = ((u64)j * (g % two_n)) % two_n;
    u64 v = a[j] % q;
    if (e < (u64)N) out[e] = v;
    else out[e - (u64)N] = v ? q - v : 0;
  }
}

/*
 * Fast base conversion (Bajard et al. 2016) of one coefficient vector from
 * basis B = {b_0..b_{nb-1}} to the prime r:
 *   Conv(x) = sum_i [x_i * (B/b_i)^-1]_{b_i} * (B/b_i mod r)   mod r
 * with the bracket the least non-negative residue.  No overflow correction.
 * in: nb limbs of N residues each (row-major).
 */
void or_base_convert(const u64* in, const u64* B, int nb, u64 r, u64* out, int N) {
  u64* hat_inv = (u64*)malloc(sizeof(u64) * (size_t)nb);  /* [(B/b_i)^-1]_{b_i} */
  u64* hat_r = (u64*)malloc(sizeof(u64) * (size_t)nb);    /* [B/b_i]_r */
  for (int i = 0; i < nb; ++i) {
    u64 prod_bi = 1 % B[i], prod_r = 1 % r;
    for (int k = 0; k < nb; ++k) {
      if (k == i) continue;
      prod_bi = or_mulmod(prod_bi, B[k] % B[i], B[i]);
      prod_r = or_mulmod(prod_r, B[k] % r, r);
    }
    hat_inv[i] = or_invmod(prod_bi, B[i]);
    hat_r[i] = prod_r;
  }
  for (int j = 0; j < N; ++j) {
    u64 acc = 0;
    for (int i = 0; i < nb; ++i) {
      u64 y = or_mulmod(in[(size_t)i * N + j] % B[i], hat_inv[i], B[i]);
      acc = addmod(acc, or_mulmod(y % r, hat_r[i], r), r);
    }
    out[j] = acc;
  }
  free(hat_inv);
  free(hat_r);
}
