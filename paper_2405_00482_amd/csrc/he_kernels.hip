// HIP kernels of the RNS-CKKS ciphertext x plaintext matrix product for gfx950.
// Residues are exact binary64 integers (fp64_mod.hpp); evaluation-domain limbs
// are stored in the orbit order of ntt_core.hpp.
// Key generation, encryption and the key-switching kernels loop over limbs
// in registers: keep their thread-index arithmetic inside the loops (see
// opaque_tid in ntt_core.hpp).
#define PVFL_OPAQUE_TID 1

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "he_dev.hpp"
#include "kernels.hpp"
#include "ntt_core.hpp"

namespace pvfl {

#define NTT_KERNEL(LOGN) __global__ __launch_bounds__(NttShape<LOGN>::T)
#define NTT_LDS(LOGN) __shared__ double s[NttShape<LOGN>::LDS]

// ---------------------------------------------------------------------------
// plain batched transforms over contiguous limbs.  Block b handles limb
// b % nl of polynomial b / nl; limb l uses prime map.idx[l].
// ---------------------------------------------------------------------------
template <int LOGN>
NTT_KERNEL(LOGN) void k_ntt_fwd(const double* __restrict__ in, double* __restrict__ out, LimbMap map, DevTabs tb) {
  constexpr int N = 1 << LOGN;
  NTT_LDS(LOGN);
  const int b = blockIdx.x, pi = map.idx[b % map.n];
  const ModQ m = tb.mods[pi];
  const double* src = in + (size_t)b * N;
  double* dst = out + (size_t)b * N;
  ntt_fwd_out<LOGN>(s, [&](int j) { return src[j]; }, tb.fwd_tw + (size_t)pi * N, tb.perm, m,
                    [&](int t, double v) { dst[t] = v; });
}

template <int LOGN>
NTT_KERNEL(LOGN) void k_ntt_inv(const double* __restrict__ in, double* __restrict__ out, LimbMap map, DevTabs tb) {
  constexpr int N = 1 << LOGN;
  NTT_LDS(LOGN);
  const int b = blockIdx.x, pi = map.idx[b % map.n];
  const ModQ m = tb.mods[pi];
  const double* src = in + (size_t)b * N;
  double* dst = out + (size_t)b * N;
  ntt_inv_in<LOGN>(s, [&](int t) { return src[t]; }, tb.inv_tw + (size_t)pi * N, tb.perm, m, tb.ninv[pi],
                   [&](int j, double v) { dst[j] = v; });
}

// signed integer coefficients [count][N] -> evaluation-domain residues
// [count][nl][N]: every limb of polynomial c is the same integer vector.
template <int LOGN>
NTT_KERNEL(LOGN) void k_import_i64(const int64_t* __restrict__ in, double* __restrict__ out, LimbMap map, DevTabs tb) {
  constexpr int N = 1 << LOGN;
  NTT_LDS(LOGN);
  const int b = blockIdx.x, c = b / map.n, pi = map.idx[b % map.n];
  const ModQ m = tb.mods[pi];
  const double t32 = tb.two32[pi];
  const int64_t* src = in + (size_t)c * N;
  double* dst = out + (size_t)b * N;
  ntt_fwd_out<LOGN>(s, [&](int j) { return i64_to_res(src[j], m, t32); }, tb.fwd_tw + (size_t)pi * N, tb.perm, m,
                    [&](int t, double v) { dst[t] = v; });
}

// The same at N <= 2^14 with one workgroup per polynomial: the integer row is
// read once, into registers, and every limb is reduced from it and
// transformed in turn, so the row's memory latency is paid once per
// polynomial instead of once per limb.
template <int LOGN>
NTT_KERNEL(LOGN) void k_import_i64_poly(const int64_t* __restrict__ in, double* __restrict__ out, LimbMap map,
                                        DevTabs tb) {
  static_assert(LOGN <= 14, "one LDS-resident limb");
  constexpr int N = 1 << LOGN, T = NttShape<LOGN>::T;
  NTT_LDS(LOGN);
  const int c = blockIdx.x;
  const int64_t* src = in + (size_t)c * N;
  // v = hi 2^32 + lo, both parts exact in binary64, split once for all limbs
  double hi[16], lo[16];
#pragma unroll
  for (int w = 0; w < 16; ++w) {
    const int64_t v = src[opaque_tid() + w * T];
    hi[w] = (double)(v >> 32);
    lo[w] = (double)(uint32_t)(v & 0xffffffffll);
  }
  for (int l = 0; l < map.n; ++l) {
    const int pi = map.idx[l];
    const ModQ m = tb.mods[pi];
    const double t32 = tb.two32[pi];
    double x[16];
#pragma unroll
    for (int w = 0; w < 16; ++w) x[w] = reduce(mulmod(reduce(hi[w], m), t32, m) + lo[w], m);  // as i64_to_res
    double* dst = out + ((size_t)c * map.n + l) * N;
    // nothing in this kernel reads the output again: stream it past L2
    ntt_fwd_regs_out<LOGN>(s, x, tb.fwd_tw + (size_t)pi * N, tb.perm, m,
                           [&](int t, double y) { __builtin_nontemporal_store(y, dst + t); });
  }
}

// evaluation-domain residues -> canonical coefficient residues as uint64
template <int LOGN>
NTT_KERNEL(LOGN) void k_export_u64(const double* __restrict__ in, uint64_t* __restrict__ out, LimbMap map, DevTabs tb) {
  constexpr int N = 1 << LOGN;
  NTT_LDS(LOGN);
  const int b = blockIdx.x, pi = map.idx[b % map.n];
  const ModQ m = tb.mods[pi];
  const double* src = in + (size_t)b * N;
  uint64_t* dst = out + (size_t)b * N;
  ntt_inv_in<LOGN>(s, [&](int t) { return src[t]; }, tb.inv_tw + (size_t)pi * N, tb.perm, m, tb.ninv[pi],
                   [&](int j, double v) { dst[j] = f64_to_u64(canon(v, m)); });
}

// The same at N <= 2^14 with one workgroup per polynomial: while one limb is
// transformed, the next limb's values are already being loaded into
// registers (its slots go to LDS only after this limb's transform is done).
template <int LOGN>
NTT_KERNEL(LOGN) void k_export_u64_poly(const double* __restrict__ in, uint64_t* __restrict__ out, LimbMap map,
                                        DevTabs tb) {
  static_assert(LOGN <= 14, "one LDS-resident limb");
  constexpr int N = 1 << LOGN, T = NttShape<LOGN>::T;
  NTT_LDS(LOGN);
  const int c = blockIdx.x;
  const double* src = in + (size_t)c * map.n * N;
  // v[2w], v[2w+1]: orbit slots t = tid + w T and t + N/2 of the current limb
  double v[16];
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    v[2 * w] = src[opaque_tid() + w * T];
    v[2 * w + 1] = src[opaque_tid() + w * T + N / 2];
  }
  for (int l = 0; l < map.n; ++l) {
    const int pi = map.idx[l];
    const ModQ m = tb.mods[pi];
    {
      OrbitWalk ow = OrbitWalk::start<LOGN>();
#pragma unroll
      for (int w = 0; w < 8; ++w) {
        const int j = ow.brv_index<LOGN>();
        s[lds_pad(j)] = reduce(v[2 * w], m);
        s[lds_pad(j ^ (N - 1))] = reduce(v[2 * w + 1], m);
        ow.next<LOGN>();
      }
    }
    if (l + 1 < map.n) {
      const double* nsrc = src + (size_t)(l + 1) * N;
#pragma unroll
      for (int w = 0; w < 8; ++w) {
        v[2 * w] = nsrc[opaque_tid() + w * T];
        v[2 * w + 1] = nsrc[opaque_tid() + w * T + N / 2];
      }
    }
    __syncthreads();
    double cf[16];
    ntt_inv_regs<LOGN>(s, cf, tb.inv_tw + (size_t)pi * N, m, tb.ninv[pi]);
    uint64_t* dst = out + ((size_t)c * map.n + l) * N;
#pragma unroll
    for (int w = 0; w < 16; ++w) __builtin_nontemporal_store(f64_to_u64(canon(cf[w], m)), dst + opaque_tid() + w * T);
    __syncthreads();  // other threads may still read this limb from LDS
  }
}

// ---------------------------------------------------------------------------
// keys and encryption
// ---------------------------------------------------------------------------
// secret key: ternary s, transformed for every prime of the context.
template <int LOGN>
NTT_KERNEL(LOGN) void k_keygen(uint64_t seed, double* __restrict__ sk, DevTabs tb) {
  constexpr int N = 1 << LOGN;
  NTT_LDS(LOGN);
  const int pi = blockIdx.x;
  const ModQ m = tb.mods[pi];
  double* dst = sk + (size_t)pi * N;
  ntt_fwd_out<LOGN>(s, [&](int j) { return (double)sample_ternary(seed, kStreamSecret, (uint64_t)j); },
                    tb.fwd_tw + (size_t)pi * N, tb.perm, m, [&](int t, double v) { dst[t] = v; });
}

// secret-key encryption of integer coefficients m (c1 = a, c0 = -a s + m + e)
// at level lv.  Block (c, i): ciphertext c, limb i; ciphertext c uses
// msg[c] and seed + c.
template <int LOGN>
NTT_KERNEL(LOGN) void k_encrypt(const int64_t* __restrict__ msg, const double* __restrict__ sk, uint64_t seed0,
                                 int lv, double* __restrict__ ct_all, double* const* __restrict__ ct_tab, DevTabs tb) {
  constexpr int N = 1 << LOGN;
  NTT_LDS(LOGN);
  const int i = blockIdx.x % (lv + 1), c = blockIdx.x / (lv + 1);
  const uint64_t seed = seed0 + (uint64_t)c;
  const int64_t* mc = msg + (size_t)c * N;
  double* ct = ct_tab ? ct_tab[c] : ct_all + (size_t)c * 2 * (lv + 1) * N;
  const ModQ m = tb.mods[i];
  const uint64_t qi = (uint64_t)m.q;
  double* c0 = ct + (size_t)i * N;
  double* c1 = ct + (size_t)(lv + 1 + i) * N;
  // a, sampled in the coefficient domain
  ntt_fwd_out<LOGN>(s, [&](int j) { return sample_uniform_res(seed, kStreamEncA | (uint64_t)i, j, qi); },
                    tb.fwd_tw + (size_t)i * N, tb.perm, m, [&](int t, double v) { c1[t] = v; });
  const double t32 = tb.two32[i];
  const double* sk_i = sk + (size_t)i * N;
  // c0 = m + e - a s; slot t of a is read back from what this thread wrote above
  ntt_fwd_out<LOGN>(s, [&](int j) {
      return reduce(i64_to_res(mc[j], m, t32) + (double)sample_cbd21(seed, kStreamEncE, (uint64_t)j), m);
    }, tb.fwd_tw + (size_t)i * N, tb.perm, m,
    [&](int t, double v) { c0[t] = reduce(v - mulmod(c1[t], sk_i[t], m), m); });
}

// public key: block i (limb i < nl): a uniform, b = -a s + e (Sec. 2.2, the
// public-key form of RLWE encryption)
template <int LOGN>
NTT_KERNEL(LOGN) void k_pk_gen(const double* __restrict__ sk, uint64_t seed, int nl, double* __restrict__ pk, DevTabs tb) {
  constexpr int N = 1 << LOGN;
  NTT_LDS(LOGN);
  const int i = blockIdx.x;
  const ModQ m = tb.mods[i];
  const uint64_t qi = (uint64_t)m.q;
  double* b = pk + (size_t)i * N;
  double* a = pk + (size_t)(nl + i) * N;
  ntt_fwd_out<LOGN>(s, [&](int j) { return sample_uniform_res(seed, kStreamPkA | (uint64_t)i, j, qi); },
                    tb.fwd_tw + (size_t)i * N, tb.perm, m, [&](int t, double v) { a[t] = v; });
  const double* sk_i = sk + (size_t)i * N;
  // slot t of a is read back from what this thread wrote above
  ntt_fwd_out<LOGN>(s, [&](int j) { return (double)sample_cbd21(seed, kStreamPkE, (uint64_t)j); },
                    tb.fwd_tw + (size_t)i * N, tb.perm, m,
                    [&](int t, double v) { b[t] = reduce(v - mulmod(a[t], sk_i[t], m), m); });
}

// public-key encryption of integer coefficients m at level lv: v ternary,
// c0 = v b + m + e0, c1 = v a + e1.  Block (c, i): ciphertext c (seed + c), limb i.
template <int LOGN>
NTT_KERNEL(LOGN) void k_encrypt_pk(const int64_t* __restrict__ msg, const double* __restrict__ pk, int pk_nl,
                                    uint64_t seed0, int lv, double* __restrict__ ct_all, DevTabs tb) {
  constexpr int N = 1 << LOGN;
  NTT_LDS(LOGN);
  const int i = blockIdx.x % (lv + 1), c = blockIdx.x / (lv + 1);
  const uint64_t seed = seed0 + (uint64_t)c;
  const int64_t* mc = msg + (size_t)c * N;
  double* ct = ct_all + (size_t)c * 2 * (lv + 1) * N;
  const ModQ m = tb.mods[i];
  double* c0 = ct + (size_t)i * N;
  double* c1 = ct + (size_t)(lv + 1 + i) * N;
  const double* b = pk + (size_t)i * N;
  const double* a = pk + (size_t)(pk_nl + i) * N;
  // v in the evaluation domain, parked in c1; every later read of slot t is by
  // the thread that wrote it
  ntt_fwd_out<LOGN>(s, [&](int j) { return (double)sample_ternary(seed, kStreamPkV, (uint64_t)j); },
                    tb.fwd_tw + (size_t)i * N, tb.perm, m, [&](int t, double v) { c1[t] = v; });
  const double t32 = tb.two32[i];
  ntt_fwd_out<LOGN>(s, [&](int j) {
      return reduce(i64_to_res(mc[j], m, t32) + (double)sample_cbd21(seed, kStreamPkE0, (uint64_t)j), m);
    }, tb.fwd_tw + (size_t)i * N, tb.perm, m,
    [&](int t, double v) { c0[t] = reduce(v + mulmod(c1[t], b[t], m), m); });
  ntt_fwd_out<LOGN>(s, [&](int j) { return (double)sample_cbd21(seed, kStreamPkE1, (uint64_t)j); },
                    tb.fwd_tw + (size_t)i * N, tb.perm, m,
                    [&](int t, double v) { c1[t] = reduce(v + mulmod(c1[t], a[t], m), m); });
}

// c0 + c1 s -> canonical coefficient residues (uint64), block i = limb i
template <int LOGN>
NTT_KERNEL(LOGN) void k_decrypt_u64(const double* __restrict__ ct, const double* __restrict__ sk, int lv,
                                     uint64_t* __restrict__ out, DevTabs tb) {
  constexpr int N = 1 << LOGN;
  NTT_LDS(LOGN);
  const int i = blockIdx.x;
  const ModQ m = tb.mods[i];
  const double* c0 = ct + (size_t)i * N;
  const double* c1 = ct + (size_t)(lv + 1 + i) * N;
  const double* sk_i = sk + (size_t)i * N;
  uint64_t* dst = out + (size_t)i * N;
  ntt_inv_in<LOGN>(s, [&](int t) { return c0[t] + mulmod(c1[t], sk_i[t], m); }, tb.inv_tw + (size_t)i * N, tb.perm,
                   m, tb.ninv[i], [&](int j, double v) { dst[j] = f64_to_u64(canon(v, m)); });
}

// c0 + c1 s -> canonical coefficient residues (binary64), for the CRT decoder;
// block (c, i) = ciphertext c, limb i
template <int LOGN>
NTT_KERNEL(LOGN) void k_decrypt_f64(const double* __restrict__ ct, const double* const* __restrict__ ct_tab,
                                     const double* __restrict__ sk, int lv, double* __restrict__ out, DevTabs tb) {
  constexpr int N = 1 << LOGN;
  NTT_LDS(LOGN);
  const int i = blockIdx.x % (lv + 1), c = blockIdx.x / (lv + 1);
  const ModQ m = tb.mods[i];
  const double* base = ct_tab ? ct_tab[c] : ct + (size_t)c * 2 * (lv + 1) * N;
  const double* c0 = base + (size_t)i * N;
  const double* c1 = base + (size_t)(lv + 1 + i) * N;
  const double* sk_i = sk + (size_t)i * N;
  double* dst = out + ((size_t)c * (lv + 1) + i) * N;
  ntt_inv_in<LOGN>(s, [&](int t) { return c0[t] + mulmod(c1[t], sk_i[t], m); }, tb.inv_tw + (size_t)i * N, tb.perm,
                   m, tb.ninv[i], [&](int j, double v) { dst[j] = canon(v, m); });
}

// Rotation (Galois) keys.  Block = (key kk, digit j, limb r of Q_L u P):
//   a uniform (coefficient domain) -> NTT;  b = -a s + e_j + [r in D_j] P phi_g(s)
// with phi_g(s) read as an orbit shift of the transformed secret.
// Layout: keys[kk][j][0 = b | 1 = a][r][N].
template <int LOGN>
NTT_KERNEL(LOGN) void k_rotkey_gen(const double* __restrict__ sk, RotKeyList list, uint64_t seed, RotKeyArgs ka,
                                    double* __restrict__ keys, DevTabs tb) {
  constexpr int N = 1 << LOGN;
  NTT_LDS(LOGN);
  const int nlimb = ka.n_limbs;
  const int r = blockIdx.x % nlimb;
  const int j = (blockIdx.x / nlimb) % ka.beta;
  const int kk = blockIdx.x / (nlimb * ka.beta);
  const ModQ m = tb.mods[r];  // limbs of Q_L u P are exactly the context's prime order
  const uint64_t g = list.galois[kk];
  const int rot = list.rot[kk];
  const uint64_t sa = kStreamKeyA | ((uint64_t)j << 40) | ((uint64_t)r << 24) | g;
  const uint64_t se = kStreamKeyE | ((uint64_t)j << 40) | g;
  double* kb = keys + ((((size_t)kk * ka.beta + j) * 2 + 0) * nlimb + r) * N;
  double* kaout = keys + ((((size_t)kk * ka.beta + j) * 2 + 1) * nlimb + r) * N;
  ntt_fwd_out<LOGN>(s, [&](int k) { return sample_uniform_res(seed, sa, k, (uint64_t)m.q); },
                    tb.fwd_tw + (size_t)r * N, tb.perm, m, [&](int t, double v) { kaout[t] = v; });
  const double* sk_r = sk + (size_t)r * N;
  const bool in_digit = (r < ka.n_q) && (r / ka.alpha == j);
  const double pmod = ka.P_mod[r];
  const int half = N / 2;
  // b = e - a s (+ P phi_g(s) on the digit's own limbs); a read back from this thread's writes
  ntt_fwd_out<LOGN>(s, [&](int k) { return (double)sample_cbd21(seed, se, (uint64_t)k); }, tb.fwd_tw + (size_t)r * N,
                    tb.perm, m, [&](int t, double e) {
                      double v = e - mulmod(kaout[t], sk_r[t], m);
                      if (in_digit) v += mulmod(pmod, sk_r[orbit_shift(t, rot, half)], m);
                      kb[t] = reduce(v, m);
                    });
}

// ---------------------------------------------------------------------------
// ModUp (hoisted once per input ciphertext).  Input ciphertext c of a batch
// is at ct + c*ct_stride; its digits go to digits + c*dig_stride.
// step 1: INTT of every limb of c1; y_i = [x_i * (Q_j/q_i)^-1]_{q_i} (canonical)
// step 2: per (digit j, target limb r not in D_j):
//         Conv = sum_{i in D_j} y_i [Q_j/q_i]_r  -> NTT -> digits[j][r]
// ---------------------------------------------------------------------------
template <int LOGN>
NTT_KERNEL(LOGN) void k_modup_intt(const double* __restrict__ ct, const double* const* __restrict__ ct_tab,
                                    size_t ct_stride, int lv, const KsLevel* __restrict__ kl, double* __restrict__ y,
                                    DevTabs tb) {
  constexpr int N = 1 << LOGN;
  NTT_LDS(LOGN);
  const int i = blockIdx.x % (lv + 1), c = blockIdx.x / (lv + 1);
  const ModQ m = tb.mods[i];
  const double* c1 = (ct_tab ? ct_tab[c] : ct + (size_t)c * ct_stride) + (size_t)(lv + 1 + i) * N;
  const double ih = kl->up_inv_hat[i];
  double* dst = y + ((size_t)c * (lv + 1) + i) * N;
  ntt_inv_in<LOGN>(s, [&](int t) { return c1[t]; }, tb.inv_tw + (size_t)i * N, tb.perm, m, tb.ninv[i],
                   [&](int j, double v) { dst[j] = canon(mulmod(canon(v, m), ih, m), m); });
}

template <int LOGN>
NTT_KERNEL(LOGN) void k_modup_conv(const double* __restrict__ y, const double* __restrict__ ct,
                                    const double* const* __restrict__ ct_tab, size_t ct_stride,
                                    const KsLevel* __restrict__ kl, double* __restrict__ digits, size_t dig_stride,
                                    DevTabs tb) {
  constexpr int N = 1 << LOGN, T = NttShape<LOGN>::T;
  NTT_LDS(LOGN);
  const int nt = kl->n_tasks;
  const KsTask task = kl->up_task[blockIdx.x % nt];
  const int c = blockIdx.x / nt;
  const int K = kl->K, lv = kl->lv;
  const int pi = task.prime;
  const ModQ m = tb.mods[pi];
  double* dst = digits + (size_t)c * dig_stride + ((size_t)task.digit * K + task.limb) * N;
  if (task.nsrc == 0) {  // limb of the digit itself: residues kept as they are
    const double* src = (ct_tab ? ct_tab[c] : ct + (size_t)c * ct_stride) + (size_t)(lv + 1 + task.limb) * N;
    for (int t = threadIdx.x; t < N; t += T) dst[t] = src[t];
    return;
  }
  const double* yc = y + (size_t)c * (lv + 1) * N;
  ntt_fwd_out<LOGN>(s, [&](int j) {
      double acc = 0.0;
      for (int u = 0; u < task.nsrc; ++u) acc += mulmod(yc[(size_t)(task.src0 + u) * N + j], task.hat[u], m);
      return reduce(acc, m);
    }, tb.fwd_tw + (size_t)pi * N, tb.perm, m, [&](int t, double v) { dst[t] = v; });
}

// ---------------------------------------------------------------------------
// ModDown Q_l u P -> Q_l with coefficient-wise rounding, on `npoly` polys
// stored [npoly][K][N] (evaluation domain); output [npoly][l+1][N].
// step 1 (P limbs): INTT, add floor(P/2), y_k = [x_k (P/p_k)^-1]_{p_k}
// step 2 (Q limbs): t_i = Conv_{P->q_i}(y) - floor(P/2) (coefficient domain)
//                   -> NTT -> out_i = (u_i - t_i) * P^-1 mod q_i
// ---------------------------------------------------------------------------
template <int LOGN>
NTT_KERNEL(LOGN) void k_moddown_p(const double* __restrict__ u, const KsLevel* __restrict__ kl,
                                   double* __restrict__ y, DevTabs tb) {
  constexpr int N = 1 << LOGN;
  NTT_LDS(LOGN);
  const int alpha = kl->alpha, K = kl->K, lv = kl->lv;
  const int k = blockIdx.x % alpha, x = blockIdx.x / alpha;
  const int pi = kl->n_q_total + k;
  const ModQ m = tb.mods[pi];
  const double* src = u + ((size_t)x * K + lv + 1 + k) * N;
  const double h = kl->down_half[lv + 1 + k];
  const double ih = kl->down_inv_hat[k];
  double* dst = y + ((size_t)x * alpha + k) * N;
  ntt_inv_in<LOGN>(s, [&](int t) { return src[t]; }, tb.inv_tw + (size_t)pi * N, tb.perm, m, tb.ninv[pi],
                   [&](int c, double v) { dst[c] = canon(mulmod(canon(v + h, m), ih, m), m); });
}

template <int LOGN>
NTT_KERNEL(LOGN) void k_moddown_q(const double* __restrict__ u, const double* __restrict__ y,
                                   const KsLevel* __restrict__ kl, double* __restrict__ out,
                                   double* const* __restrict__ out_tab, DevTabs tb) {
  constexpr int N = 1 << LOGN;
  NTT_LDS(LOGN);
  const int alpha = kl->alpha, K = kl->K, lv = kl->lv;
  const int i = blockIdx.x % (lv + 1), x = blockIdx.x / (lv + 1);
  const ModQ m = tb.mods[i];
  const double h = kl->down_half[i];
  const double* yx = y + (size_t)x * alpha * N;
  const double pinv = kl->down_pinv[i];
  const double* ui = u + ((size_t)x * K + i) * N;
  double* oi = out_tab ? out_tab[x >> 1] + ((size_t)(x & 1) * (lv + 1) + i) * N : out + ((size_t)x * (lv + 1) + i) * N;
  ntt_fwd_out<LOGN>(s, [&](int c) {
      double acc = -h;
      for (int k = 0; k < alpha; ++k) acc += mulmod(yx[(size_t)k * N + c], kl->down_hat[k * kMaxLimbs + i], m);
      return reduce(acc, m);
    }, tb.fwd_tw + (size_t)i * N, tb.perm, m, [&](int t, double v) { oi[t] = reduce(mulmod(ui[t] - v, pinv, m), m); });
}

// Rescale by q_lv (drop the last limb, coefficient-wise rounding) on `npoly`
// polys [npoly][lv+1][N] -> [npoly][lv][N].  Same formula as ModDown with P = q_lv.
template <int LOGN>
NTT_KERNEL(LOGN) void k_rescale(const double* __restrict__ in, int lv, const RescaleArgs ra, double* __restrict__ out,
                                 DevTabs tb) {
  constexpr int N = 1 << LOGN, PER = NttShape<LOGN>::PER;
  NTT_LDS(LOGN);
  const int i = blockIdx.x % lv, x = blockIdx.x / lv;
  const ModQ ml = tb.mods[lv];
  const ModQ m = tb.mods[i];
  // INTT of the dropped limb (every block recomputes it; the limb is L2-resident)
  const double* last = in + ((size_t)x * (lv + 1) + lv) * N;
  double c[PER];
  ntt_inv_in_regs<LOGN>(s, [&](int t) { return last[t]; }, tb.inv_tw + (size_t)lv * N, tb.perm, ml, tb.ninv[lv], c);
  const double hl = ra.half_mod_last, hi = ra.half_mod[i];
  // [c + h]_{q_l} lifted to q_i, minus h mod q_i
#pragma unroll
  for (int w = 0; w < PER; ++w) c[w] = reduce(canon(c[w] + hl, ml) - hi, m);
  const double inv = ra.inv_last[i];
  const double* ui = in + ((size_t)x * (lv + 1) + i) * N;
  double* oi = out + ((size_t)x * lv + i) * N;
  ntt_fwd_regs_out<LOGN>(s, c, tb.fwd_tw + (size_t)i * N, tb.perm, m,
                         [&](int t, double v) { oi[t] = reduce(mulmod(ui[t] - v, inv, m), m); });
}

// ---------------------------------------------------------------------------
// The hot loop: fused hoisted rotations x plaintext diagonals, lazy ModDown.
//   acc0 = sum_i pt_i * (P phi_i(c0) + sum_j phi_i(D_j) b_{i,j})
//   acc1 = sum_i pt_i * (               sum_j phi_i(D_j) a_{i,j})
// over Q_l u P; the i = 0 term is pt_0 * (P c0, P c1) on the Q limbs.
// Thread = (limb r, coefficient t); blockIdx.z splits the diagonals into
// chunks whose partial sums go to part[z][2][K][N].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_diag_lazy(DiagArgs a) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y;
  const int N = a.N, half = N >> 1, K = a.K;
  const int pi = a.limb_prime[r];
  const int klimb = a.key_limb[r];
  const bool isq = r <= a.lv;
  const ModQ m = a.mods[pi];
  const int i0 = blockIdx.z * a.chunk;
  const int i1 = min(i0 + a.chunk, a.mprime);
  double acc0 = 0.0, acc1 = 0.0;
  const size_t limbN = (size_t)r * N;
  int cnt = 0;
  for (int i = i0; i < i1; ++i) {
    const double p = a.pt[(size_t)a.pt_index[i] * K * N + limbN + t];
    if (a.rot[i] == 0) {
      if (isq) {
        acc0 += mulmod(p, a.pc[limbN + t], m);
        acc1 += mulmod(p, a.pc[(size_t)(a.lv + 1) * N + limbN + t], m);
      }
    } else {
      const int ts = orbit_shift(t, a.rot[i], half);
      const double* key = a.keys + (size_t)a.slot_of_rot[a.rot[i]] * a.key_stride;
      double u0 = 0.0, u1 = 0.0;
      for (int j = 0; j < a.beta; ++j) {
        const double d = a.digits[((size_t)j * K) * N + limbN + ts];
        const double* kj = key + (size_t)j * 2 * a.key_limbs * N;
        u0 += mulmod(d, kj[(size_t)klimb * N + t], m);
        u1 += mulmod(d, kj[(size_t)(a.key_limbs + klimb) * N + t], m);
      }
      if (isq) u0 += a.pc[limbN + ts];
      acc0 += mulmod(p, u0, m);
      acc1 += mulmod(p, u1, m);
    }
    if (++cnt == 8) { acc0 = reduce(acc0, m); acc1 = reduce(acc1, m); cnt = 0; }
  }
  double* part = a.part + (size_t)blockIdx.z * 2 * K * N;
  part[limbN + t] = reduce(acc0, m);
  part[(size_t)K * N + limbN + t] = reduce(acc1, m);
}

// sum the chunk partials of every group y: part[y][nchunk][2][K][N] -> acc[y][2][K][N]
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ part, int nchunk, int K, int N,
                                                       LimbMap limb_prime, const ModQ* __restrict__ mods,
                                                       double* __restrict__ acc) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t tot = (size_t)2 * K * N;
  if (idx >= tot) return;
  part += (size_t)blockIdx.y * nchunk * tot;
  acc += (size_t)blockIdx.y * tot;
  const int r = (int)((idx / N) % K);
  const ModQ m = mods[limb_prime.idx[r]];
  double v = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    v += part[(size_t)c * tot + idx];
    if ((c & 7) == 7) v = reduce(v, m);
  }
  acc[idx] = reduce(v, m);
}

// P * (c0, c1) on the Q limbs, [2][lv+1][N]
__global__ __launch_bounds__(256) void k_scale_by_p(const double* __restrict__ ct, const double* const* __restrict__ ct_tab,
                                                    int lv, int N, const double* __restrict__ pmod,
                                                    const ModQ* __restrict__ mods, double* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t tot = (size_t)2 * (lv + 1) * N;
  if (idx >= tot) return;
  const int c = blockIdx.y;
  const double* src = ct_tab ? ct_tab[c] : ct + (size_t)c * tot;
  const int i = (int)((idx / N) % (lv + 1));
  out[(size_t)c * tot + idx] = reduce(mulmod(src[idx], pmod[i], mods[i]), mods[i]);
}

// ---------------------------------------------------------------------------
// element-wise ciphertext operations (evaluation domain)
// ---------------------------------------------------------------------------
// out[x][i] = in[x][i] * pt[i] for x in {0,1}; pt has >= lv+1 limbs
__global__ __launch_bounds__(256) void k_ct_mul_pt(const double* __restrict__ ct, const double* __restrict__ pt, int lv, int N,
                                                   const ModQ* __restrict__ mods, double* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t tot = (size_t)2 * (lv + 1) * N;
  if (idx >= tot) return;
  const size_t within = idx % ((size_t)(lv + 1) * N);
  const int i = (int)(within / N);
  out[idx] = mulmod(ct[idx], pt[within], mods[i]);
}

__global__ __launch_bounds__(256) void k_ct_add(const double* __restrict__ a, const double* __restrict__ b, int lv, int N,
                                                const ModQ* __restrict__ mods, double* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t tot = (size_t)2 * (lv + 1) * N;
  if (idx >= tot) return;
  const int i = (int)((idx / N) % (lv + 1));
  out[idx] = reduce(a[idx] + b[idx], mods[i]);
}

// automorphism X -> X^(5^rot) on npoly polys of nl limbs: an orbit shift
__global__ __launch_bounds__(256) void k_automorph(const double* __restrict__ in, int npoly_limbs, int N, int rot,
                                                   double* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)npoly_limbs * N) return;
  const int t = (int)(idx % N);
  out[idx] = in[idx - t + orbit_shift(t, rot, N >> 1)];
}

// (u0, u1) = sum_j D_j * (b_j, a_j) over K limbs, digits optionally shifted by
// `rot` (hoisted rotation) -- the unfused key inner product of the eager plan.
__global__ __launch_bounds__(256) void k_key_inner(const double* __restrict__ digits, int beta, int K, int N, int rot,
                                                   const double* __restrict__ key, int key_limbs,
                                                   LimbMap limb_prime, LimbMap key_limb,
                                                   const ModQ* __restrict__ mods, double* __restrict__ u) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y;
  const ModQ m = mods[limb_prime.idx[r]];
  const int ts = orbit_shift(t, rot, N >> 1);
  const int kl = key_limb.idx[r];
  double u0 = 0.0, u1 = 0.0;
  for (int j = 0; j < beta; ++j) {
    const double d = digits[((size_t)j * K + r) * N + ts];
    const double* kj = key + (size_t)j * 2 * key_limbs * N;
    u0 += mulmod(d, kj[(size_t)kl * N + t], m);
    u1 += mulmod(d, kj[(size_t)(key_limbs + kl) * N + t], m);
  }
  u[(size_t)r * N + t] = reduce(u0, m);
  u[(size_t)(K + r) * N + t] = reduce(u1, m);
}

__global__ __launch_bounds__(256) void k_fill_zero(double* __restrict__ p, size_t n) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx < n) p[idx] = 0.0;
}

__global__ __launch_bounds__(256) void k_add_limbs(const double* __restrict__ a, const double* __restrict__ b, int nlimbs,
                                                   int N, LimbMap map, const ModQ* __restrict__ mods,
                                                   double* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)nlimbs * N) return;
  const int l = (int)(idx / N) % map.n;
  out[idx] = reduce(a[idx] + b[idx], mods[map.idx[l]]);
}

// one term of the eager (per-rotation ModDown) plan:
//   acc0 += (c0[shift] + v0) * pt,  acc1 += v1 * pt      (v != null)
//   acc0 += c0 * pt,                acc1 += c1 * pt      (v == null)
__global__ __launch_bounds__(256) void k_eager_term(const double* __restrict__ c0, const double* __restrict__ c1,
                                                    const double* __restrict__ v, int rot, const double* __restrict__ pt,
                                                    int lv, int N, const ModQ* __restrict__ mods, double* __restrict__ acc) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t Q = (size_t)(lv + 1) * N;
  if (idx >= Q) return;
  const int i = (int)(idx / N), t = (int)(idx % N);
  const ModQ m = mods[i];
  const double p = pt[idx];
  double x0, x1;
  if (v) {
    x0 = reduce(c0[idx - t + orbit_shift(t, rot, N >> 1)] + v[idx], m);
    x1 = v[Q + idx];
  } else {
    x0 = c0[idx];
    x1 = c1[idx];
  }
  acc[idx] = reduce(acc[idx] + mulmod(x0, p, m), m);
  acc[Q + idx] = reduce(acc[Q + idx] + mulmod(x1, p, m), m);
}

// Alg. 3 ciphertext-matrix product: thread = (coefficient t, limb r, output k)
__global__ __launch_bounds__(256) void k_ctmat(const double* __restrict__ ct, const double* __restrict__ pt, int nct,
                                               int nout, int lv, int N, const ModQ* __restrict__ mods,
                                               double* __restrict__ out) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y, k = blockIdx.z;
  const ModQ m = mods[r];
  const size_t Q = (size_t)(lv + 1) * N;
  const size_t off = (size_t)r * N + t;
  double a0 = 0.0, a1 = 0.0;
  for (int i = 0; i < nct; ++i) {
    const double p = pt[((size_t)i * nout + k) * Q + off];
    a0 += mulmod(ct[(size_t)i * 2 * Q + off], p, m);
    a1 += mulmod(ct[(size_t)i * 2 * Q + Q + off], p, m);
    if ((i & 7) == 7) { a0 = reduce(a0, m); a1 = reduce(a1, m); }
  }
  out[(size_t)k * 2 * Q + off] = reduce(a0, m);
  out[(size_t)k * 2 * Q + Q + off] = reduce(a1, m);
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <int LOGN>
static void launch_ntt_all(const LaunchCtx& L, NttOp op, const void* in, void* out, int nblocks, LimbMap map) {
  const dim3 grid(nblocks), block(NttShape<LOGN>::T);
  switch (op) {
    case NttOp::Fwd: hipLaunchKernelGGL(k_ntt_fwd<LOGN>, grid, block, 0, L.stream, (const double*)in, (double*)out, map, L.tb); break;
    case NttOp::Inv: hipLaunchKernelGGL(k_ntt_inv<LOGN>, grid, block, 0, L.stream, (const double*)in, (double*)out, map, L.tb); break;
    case NttOp::ImportI64:
      if constexpr (LOGN <= 14)  // one workgroup per polynomial (nblocks = polynomials x limbs)
        hipLaunchKernelGGL(k_import_i64_poly<LOGN>, dim3(nblocks / map.n), block, 0, L.stream, (const int64_t*)in,
                           (double*)out, map, L.tb);
      else
        hipLaunchKernelGGL(k_import_i64<LOGN>, grid, block, 0, L.stream, (const int64_t*)in, (double*)out, map, L.tb);
      break;
    case NttOp::ExportU64:
      if constexpr (LOGN <= 14)  // one workgroup per polynomial (nblocks = polynomials x limbs)
        hipLaunchKernelGGL(k_export_u64_poly<LOGN>, dim3(nblocks / map.n), block, 0, L.stream, (const double*)in,
                           (uint64_t*)out, map, L.tb);
      else
        hipLaunchKernelGGL(k_export_u64<LOGN>, grid, block, 0, L.stream, (const double*)in, (uint64_t*)out, map, L.tb);
      break;
  }
}

#define DISPATCH_LOGN(L, FN, ...)                         \
  switch ((L).logN) {                                     \
    case 12: FN<12>(__VA_ARGS__); break;                  \
    case 13: FN<13>(__VA_ARGS__); break;                  \
    case 14: FN<14>(__VA_ARGS__); break;                  \
    case 15: FN<15>(__VA_ARGS__); break;                  \
    default: return hipErrorInvalidValue;                 \
  }

hipError_t launch_ntt(const LaunchCtx& L, NttOp op, const void* in, void* out, int nblocks, LimbMap map) {
  if (nblocks <= 0) return hipSuccess;
  DISPATCH_LOGN(L, launch_ntt_all, L, op, in, out, nblocks, map);
  return hipGetLastError();
}

template <int LOGN>
static void keygen_impl(const LaunchCtx& L, uint64_t seed, double* sk, int n_mod) {
  hipLaunchKernelGGL(k_keygen<LOGN>, dim3(n_mod), dim3(NttShape<LOGN>::T), 0, L.stream, seed, sk, L.tb);
}
hipError_t launch_keygen(const LaunchCtx& L, uint64_t seed, double* sk, int n_mod) {
  DISPATCH_LOGN(L, keygen_impl, L, seed, sk, n_mod);
  return hipGetLastError();
}

template <int LOGN>
static void pk_gen_impl(const LaunchCtx& L, const double* sk, uint64_t seed, int nl, double* pk) {
  hipLaunchKernelGGL(k_pk_gen<LOGN>, dim3(nl), dim3(NttShape<LOGN>::T), 0, L.stream, sk, seed, nl, pk, L.tb);
}
hipError_t launch_pk_gen(const LaunchCtx& L, const double* sk, uint64_t seed, int nl, double* pk) {
  DISPATCH_LOGN(L, pk_gen_impl, L, sk, seed, nl, pk);
  return hipGetLastError();
}
template <int LOGN>
static void encrypt_pk_impl(const LaunchCtx& L, const int64_t* msg, int nct, const double* pk, int pk_nl, uint64_t seed,
                            int lv, double* ct) {
  hipLaunchKernelGGL(k_encrypt_pk<LOGN>, dim3(nct * (lv + 1)), dim3(NttShape<LOGN>::T), 0, L.stream, msg, pk, pk_nl,
                     seed, lv, ct, L.tb);
}
hipError_t launch_encrypt_pk(const LaunchCtx& L, const int64_t* msg, int nct, const double* pk, int pk_nl,
                             uint64_t seed, int lv, double* ct) {
  if (nct <= 0) return hipSuccess;
  DISPATCH_LOGN(L, encrypt_pk_impl, L, msg, nct, pk, pk_nl, seed, lv, ct);
  return hipGetLastError();
}

template <int LOGN>
static void encrypt_impl(const LaunchCtx& L, const int64_t* msg, int nct, const double* sk, uint64_t seed, int lv,
                         double* ct, double* const* ct_tab) {
  hipLaunchKernelGGL(k_encrypt<LOGN>, dim3(nct * (lv + 1)), dim3(NttShape<LOGN>::T), 0, L.stream, msg, sk, seed, lv, ct,
                     ct_tab, L.tb);
}
hipError_t launch_encrypt(const LaunchCtx& L, const int64_t* msg, int nct, const double* sk, uint64_t seed, int lv,
                          double* ct, double* const* ct_tab) {
  if (nct <= 0) return hipSuccess;
  DISPATCH_LOGN(L, encrypt_impl, L, msg, nct, sk, seed, lv, ct, ct_tab);
  return hipGetLastError();
}

template <int LOGN>
static void decrypt_u64_impl(const LaunchCtx& L, const double* ct, const double* sk, int lv, uint64_t* out) {
  hipLaunchKernelGGL(k_decrypt_u64<LOGN>, dim3(lv + 1), dim3(NttShape<LOGN>::T), 0, L.stream, ct, sk, lv, out, L.tb);
}
hipError_t launch_decrypt_u64(const LaunchCtx& L, const double* ct, const double* sk, int lv, uint64_t* out) {
  DISPATCH_LOGN(L, decrypt_u64_impl, L, ct, sk, lv, out);
  return hipGetLastError();
}

template <int LOGN>
static void decrypt_f64_impl(const LaunchCtx& L, const double* ct, const double* const* ct_tab, int nct, const double* sk,
                             int lv, double* out) {
  hipLaunchKernelGGL(k_decrypt_f64<LOGN>, dim3(nct * (lv + 1)), dim3(NttShape<LOGN>::T), 0, L.stream, ct, ct_tab, sk, lv,
                     out, L.tb);
}
hipError_t launch_decrypt_f64(const LaunchCtx& L, const double* ct, int nct, const double* sk, int lv, double* out,
                              const double* const* ct_tab) {
  DISPATCH_LOGN(L, decrypt_f64_impl, L, ct, ct_tab, nct, sk, lv, out);
  return hipGetLastError();
}

template <int LOGN>
static void rotkey_impl(const LaunchCtx& L, const double* sk, const RotKeyList& list, int nkeys, uint64_t seed,
                        const RotKeyArgs& ka, double* keys) {
  hipLaunchKernelGGL(k_rotkey_gen<LOGN>, dim3(nkeys * ka.beta * ka.n_limbs), dim3(NttShape<LOGN>::T), 0, L.stream,
                     sk, list, seed, ka, keys, L.tb);
}
hipError_t launch_rotkey_gen(const LaunchCtx& L, const double* sk, const RotKeyList& list, int nkeys, uint64_t seed,
                             const RotKeyArgs& ka, double* keys) {
  if (nkeys <= 0) return hipSuccess;
  if (nkeys > kKeysPerLaunch) return hipErrorInvalidValue;
  DISPATCH_LOGN(L, rotkey_impl, L, sk, list, nkeys, seed, ka, keys);
  return hipGetLastError();
}

template <int LOGN>
static void modup_impl(const LaunchCtx& L, const double* ct, const double* const* ct_tab, size_t ct_stride, int nct,
                       int lv, const KsLevel* kl_dev, int n_tasks, double* y, double* digits, size_t dig_stride) {
  hipLaunchKernelGGL(k_modup_intt<LOGN>, dim3(nct * (lv + 1)), dim3(NttShape<LOGN>::T), 0, L.stream, ct, ct_tab, ct_stride,
                     lv, kl_dev, y, L.tb);
  hipLaunchKernelGGL(k_modup_conv<LOGN>, dim3(nct * n_tasks), dim3(NttShape<LOGN>::T), 0, L.stream, y, ct, ct_tab,
                     ct_stride, kl_dev, digits, dig_stride, L.tb);
}
hipError_t launch_modup(const LaunchCtx& L, const double* ct, size_t ct_stride, int nct, int lv, const KsLevel* kl_dev,
                        int n_tasks, double* y, double* digits, size_t dig_stride, const double* const* ct_tab) {
  if (nct <= 0) return hipSuccess;
  DISPATCH_LOGN(L, modup_impl, L, ct, ct_tab, ct_stride, nct, lv, kl_dev, n_tasks, y, digits, dig_stride);
  return hipGetLastError();
}

template <int LOGN>
static void moddown_impl(const LaunchCtx& L, const double* u, int npoly, int lv, int alpha, const KsLevel* kl_dev,
                         double* y, double* out, double* const* out_tab) {
  hipLaunchKernelGGL(k_moddown_p<LOGN>, dim3(npoly * alpha), dim3(NttShape<LOGN>::T), 0, L.stream, u, kl_dev, y, L.tb);
  hipLaunchKernelGGL(k_moddown_q<LOGN>, dim3(npoly * (lv + 1)), dim3(NttShape<LOGN>::T), 0, L.stream, u, y, kl_dev, out,
                     out_tab, L.tb);
}
hipError_t launch_moddown(const LaunchCtx& L, const double* u, int npoly, int lv, int alpha, const KsLevel* kl_dev,
                          double* y, double* out, double* const* out_tab) {
  DISPATCH_LOGN(L, moddown_impl, L, u, npoly, lv, alpha, kl_dev, y, out, out_tab);
  return hipGetLastError();
}

template <int LOGN>
static void rescale_impl(const LaunchCtx& L, const double* in, int npoly, int lv, const RescaleArgs& ra, double* out) {
  hipLaunchKernelGGL(k_rescale<LOGN>, dim3(npoly * lv), dim3(NttShape<LOGN>::T), 0, L.stream, in, lv, ra, out, L.tb);
}
hipError_t launch_rescale(const LaunchCtx& L, const double* in, int npoly, int lv, const RescaleArgs& ra, double* out) {
  DISPATCH_LOGN(L, rescale_impl, L, in, npoly, lv, ra, out);
  return hipGetLastError();
}

static inline unsigned blocks_for(size_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_diag_lazy(const LaunchCtx& L, const DiagArgs& a, int nchunk) {
  const dim3 grid(a.N / 256, a.K, nchunk);
  hipLaunchKernelGGL(k_diag_lazy, grid, dim3(256), 0, L.stream, a);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const LaunchCtx& L, const double* part, int nchunk, int K, int N, LimbMap limb_prime,
                               double* acc, int ngroups) {
  const size_t tot = (size_t)2 * K * N;
  if (ngroups < 1) return hipSuccess;
  hipLaunchKernelGGL(k_sum_partials, dim3(blocks_for(tot), ngroups), dim3(256), 0, L.stream, part, nchunk, K, N,
                     limb_prime, L.tb.mods, acc);
  return hipGetLastError();
}

hipError_t launch_ctmat(const LaunchCtx& L, const double* ct, const double* pt, int nct, int nout, int lv, int N,
                        double* out) {
  hipLaunchKernelGGL(k_ctmat, dim3(N / 256, lv + 1, nout), dim3(256), 0, L.stream, ct, pt, nct, nout, lv, N, L.tb.mods,
                     out);
  return hipGetLastError();
}

hipError_t launch_fill_zero(const LaunchCtx& L, double* p, size_t n) {
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks_for(n)), dim3(256), 0, L.stream, p, n);
  return hipGetLastError();
}

hipError_t launch_add_limbs(const LaunchCtx& L, const double* a, const double* b, int nlimbs, int N, LimbMap map,
                            double* out) {
  const size_t tot = (size_t)nlimbs * N;
  hipLaunchKernelGGL(k_add_limbs, dim3(blocks_for(tot)), dim3(256), 0, L.stream, a, b, nlimbs, N, map, L.tb.mods, out);
  return hipGetLastError();
}

hipError_t launch_eager_term(const LaunchCtx& L, const double* c0, const double* c1, const double* v, int rot,
                             const double* pt, int lv, int N, double* acc) {
  const size_t tot = (size_t)(lv + 1) * N;
  hipLaunchKernelGGL(k_eager_term, dim3(blocks_for(tot)), dim3(256), 0, L.stream, c0, c1, v, rot, pt, lv, N, L.tb.mods,
                     acc);
  return hipGetLastError();
}

hipError_t launch_scale_by_p(const LaunchCtx& L, const double* ct, int lv, int N, const double* pmod_dev, double* out,
                             int nct, const double* const* ct_tab) {
  const size_t tot = (size_t)2 * (lv + 1) * N;
  hipLaunchKernelGGL(k_scale_by_p, dim3(blocks_for(tot), nct), dim3(256), 0, L.stream, ct, ct_tab, lv, N, pmod_dev,
                     L.tb.mods, out);
  return hipGetLastError();
}

hipError_t launch_ct_mul_pt(const LaunchCtx& L, const double* ct, const double* pt, int lv, int N, double* out) {
  const size_t tot = (size_t)2 * (lv + 1) * N;
  hipLaunchKernelGGL(k_ct_mul_pt, dim3(blocks_for(tot)), dim3(256), 0, L.stream, ct, pt, lv, N, L.tb.mods, out);
  return hipGetLastError();
}

hipError_t launch_ct_add(const LaunchCtx& L, const double* a, const double* b, int lv, int N, double* out) {
  const size_t tot = (size_t)2 * (lv + 1) * N;
  hipLaunchKernelGGL(k_ct_add, dim3(blocks_for(tot)), dim3(256), 0, L.stream, a, b, lv, N, L.tb.mods, out);
  return hipGetLastError();
}

hipError_t launch_automorph(const LaunchCtx& L, const double* in, int npoly_limbs, int N, int rot, double* out) {
  const size_t tot = (size_t)npoly_limbs * N;
  hipLaunchKernelGGL(k_automorph, dim3(blocks_for(tot)), dim3(256), 0, L.stream, in, npoly_limbs, N, rot, out);
  return hipGetLastError();
}

hipError_t launch_key_inner(const LaunchCtx& L, const double* digits, int beta, int K, int N, int rot, const double* key,
                            int key_limbs, LimbMap limb_prime, LimbMap key_limb, double* u) {
  hipLaunchKernelGGL(k_key_inner, dim3(N / 256, K), dim3(256), 0, L.stream, digits, beta, K, N, rot, key, key_limbs,
                     limb_prime, key_limb, L.tb.mods, u);
  return hipGetLastError();
}

}  // namespace pvfl
