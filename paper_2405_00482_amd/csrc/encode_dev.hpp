// Device helpers of the canonical-embedding encoder/decoder and the plan
// packing, shared by the single-plan and the batched kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "encode.hpp"
#include "ntt_core.hpp"

#include <type_traits>

namespace pvfl {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// padded index of complex element i in LDS (one pad slot every 16): breaks
// the bank conflicts of strided and bit-reversed access
__device__ __forceinline__ int cpad(int i) { return i + (i >> 4); }

__device__ __forceinline__ double round_half_away(double x) {
  const double r = __builtin_trunc(x + (x >= 0.0 ? 0.5 : -0.5));
  return r;
}

// S radix-2 DIF stages S0 .. S0+S-1 of the M = N/2 point FFT, on register
// sets of 2^S elements {base + u * stride} (stride = half-length of the last
// stage).  Each thread owns 8 elements (M = 8 T), i.e. 8 / 2^S sets; the sets
// partition the array, so a set is loaded, transformed and written back in
// place without a barrier in between.  At stage s a butterfly pairs elements
// half_s = M >> (s+1) apart with twiddle W_M^(j 2^s), j = index mod half_s,
// which for element u of a set is off + (u mod 2^(S-1-st)) * stride.
// A pass is wave-local when a wave's 64 threads own one contiguous run of
// 512 elements: one set of 8 per thread with a stride of at most 64.
template <int LOGN, int S, int S0>
constexpr bool fft_pass_wave_local() {
  return S == 3 && LOGN - 1 - S0 - S <= 6;
}

// Ends with a workgroup barrier, or only a wave-level LDS fence when this
// pass and the next one (NEXT_LOCAL) are both wave-local: the next pass then
// reads only what the same wave wrote.
template <int LOGN, int S, int S0, int TWSH, bool NEXT_LOCAL>
__device__ __forceinline__ void fft_pass(double2* a, const double2* __restrict__ tw, bool conj) {
  constexpr int LOGM = LOGN - 1, M = 1 << LOGM, T = NttShape<LOGN>::T;
  constexpr int SET = 1 << S, NS = 8 >> S;
  static_assert(M == 8 * T, "eight FFT points per thread");
  constexpr int LS = LOGM - S0 - S;  // log2 stride
  constexpr unsigned stride = 1u << LS;
  const unsigned tid = opaque_tid();
  if (tid < (unsigned)T) {  // a transform of M < 8 * blockDim points leaves the other threads idle
  int base[NS], off[NS];
  double2 x[8];
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const unsigned c = (unsigned)(q * T) + tid;
    off[q] = (int)(c & (stride - 1u));
    base[q] = (int)(((c >> LS) << (LS + S)) | (unsigned)off[q]);
#pragma unroll
    for (int u = 0; u < SET; ++u) x[q * SET + u] = a[cpad(base[q] + (u << LS))];
  }
#pragma unroll
  for (int st = 0; st < S; ++st) {
    const int s = S0 + st;
    const int hs = SET >> (st + 1);
#pragma unroll
    for (int q = 0; q < NS; ++q) {
#pragma unroll
      for (int u = 0; u < SET; ++u) {
        if (u & hs) continue;
        double2 w = tw[((off[q] + ((u & (hs - 1)) << LS)) << s) << TWSH];
        if (conj) w = cconj(w);
        const double2 U = x[q * SET + u], V = x[q * SET + u + hs];
        x[q * SET + u] = make_double2(U.x + V.x, U.y + V.y);
        x[q * SET + u + hs] = cmul(make_double2(U.x - V.x, U.y - V.y), w);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NS; ++q)
#pragma unroll
    for (int u = 0; u < SET; ++u) a[cpad(base[q] + (u << LS))] = x[q * SET + u];
  }
  if constexpr (fft_pass_wave_local<LOGN, S, S0>() && NEXT_LOCAL)
    wave_lds_sync();
  else
    __syncthreads();
}

// TWSH = 1 runs the 2^(LOGN-1)-point transform with the table of twice that
// size (every second entry), as the halves of the 2^15 ring's FFT do
template <int LOGN, int S0, int TWSH = 0>
__device__ __forceinline__ void fft_passes(double2* a, const double2* __restrict__ tw, bool conj) {
  constexpr int LEFT = LOGN - 1 - S0;
  if constexpr (LEFT >= 3) {
    constexpr int NLEFT = LEFT - 3;  // stages after this pass
    constexpr bool next_local = NLEFT >= 3 && fft_pass_wave_local<LOGN, 3, S0 + 3>();
    fft_pass<LOGN, 3, S0, TWSH, next_local>(a, tw, conj);
    fft_passes<LOGN, S0 + 3, TWSH>(a, tw, conj);
  } else if constexpr (LEFT > 0) {
    fft_pass<LOGN, LEFT, S0, TWSH, false>(a, tw, conj);
  }
}

// In-place DIF FFT over M = N/2 points in LDS (padded by cpad), sign -1
// (conj = false) or +1; the result is left in bit-reversed order.  The input
// must be complete in LDS (barrier before the call); the call ends with a
// barrier.  Radix-8 register passes: ceil(log2(M) / 3) LDS round trips.
template <int LOGN>
__device__ __forceinline__ void fft_dif_lds(double2* a, const double2* __restrict__ tw, bool conj) {
  static_assert(LOGN <= 14, "the 2^15 ring's FFT is split in halves (encode_to_regs, k_decode)");
  fft_passes<LOGN, 0>(a, tw, conj);
}

// Half h of the 2^15 ring's M = 2^14 point DIF FFT, already past its first
// stage and placed in LDS: stages 1.. of the full transform restricted to
// the half are a 2^13-point DIF FFT with twiddle indices doubled.
__device__ __forceinline__ void fft_dif_half15(double2* a, const double2* __restrict__ tw, bool conj) {
  fft_passes<14, 0, 1>(a, tw, conj);
}

__device__ __forceinline__ int brev(int x, int bits) { return (int)(__brev((unsigned)x) >> (32 - bits)); }

// Centred CRT lift (Garner mixed radix) of coefficient kk from its residues
// base[i N + kk], i < nl.  NL > 0 fixes the limb count at compile time, so
// the mixed-radix digits stay in registers; NL = 0 takes nl at run time.
template <int NL>
__device__ __forceinline__ double crt_lift(const double* __restrict__ base, int kk, int N, const CrtTabs& ct,
                                           int nl_rt) {
  const int nl = NL > 0 ? NL : nl_rt;
  double v[NL > 0 ? NL : kMaxLimbs];
#pragma unroll
  for (int i = 0; i < nl; ++i) {
    const ModQ m = ct.mods[i];
    double x = base[(size_t)i * N + kk];
#pragma unroll
    for (int j = 0; j < i; ++j) x = mulmod(x - v[j], ct.garner_inv[j * kMaxLimbs + i], m);
    v[i] = canon(x, m);
  }
  // sign: compare with the mixed-radix digits of (Q-1)/2 from the top
  int cmp = 0;
#pragma unroll
  for (int i = nl - 1; i >= 0; --i) {
    const double h2 = 0.5 * (ct.mods[i].q - 1.0);
    if (cmp == 0) cmp = (v[i] > h2) ? 1 : ((v[i] < h2) ? -1 : 0);
  }
  double acc = (cmp > 0) ? v[nl - 1] - ct.mods[nl - 1].q : v[nl - 1];
#pragma unroll
  for (int i = nl - 2; i >= 0; --i) acc = acc * ct.mods[i].q + v[i];
  return acc;
}

// Decode of one ciphertext's coefficient residues base[i N + k] (i < nl,
// canonical) up to the slot values, N <= 2^14: CRT lift, twist, DFT with sign
// +1; the spectrum is left in LDS (w, padded, bit-reversed order) for
// decoded_slot().  Ends with a barrier.
template <int LOGN>
__device__ __forceinline__ void decode_to_lds(const double* __restrict__ base, int nl, const CrtTabs& ct,
                                              const EncTabs& et, double2* w) {
  static_assert(LOGN <= 14, "the 2^15 ring's decode splits its FFT in halves");
  constexpr int N = 1 << LOGN, M = N / 2, T = NttShape<LOGN>::T;
  // twisted w_k = (m_k + i m_(k+N/2)) zeta^k
  auto fill = [&](auto nl_c) {
    constexpr int NL = decltype(nl_c)::value;
    for (int k = opaque_tid(); k < M; k += T)
      w[cpad(k)] = cmul(make_double2(crt_lift<NL>(base, k, N, ct, nl), crt_lift<NL>(base, k + M, N, ct, nl)),
                        et.twist[k]);
  };
  switch (nl) {  // the usual output levels get register-resident digits
    case 1: fill(std::integral_constant<int, 1>()); break;
    case 2: fill(std::integral_constant<int, 2>()); break;
    case 3: fill(std::integral_constant<int, 3>()); break;
    case 4: fill(std::integral_constant<int, 4>()); break;
    case 5: fill(std::integral_constant<int, 5>()); break;
    case 6: fill(std::integral_constant<int, 6>()); break;
    default: fill(std::integral_constant<int, 0>()); break;
  }
  __syncthreads();
  fft_dif_lds<LOGN>(w, et.fft_tw, true);
}

// slot j of the spectrum decode_to_lds left in LDS, as a cleartext value
template <int LOGN>
__device__ __forceinline__ double decoded_slot(const double2* w, const EncTabs& et, int j, double inv_scale) {
  return w[cpad(brev(et.slot2f[j], LOGN - 1))].x * inv_scale;
}

// Element of X that slot s of plaintext k holds (a KIND plan), or -1 where the
// slot is zero (padding, outside the matrix).
template <int KIND>
__device__ __forceinline__ long pt_slot_index(const EncodeArgs& a, int k, int s) {
  if constexpr (KIND == 0) {  // HYBRID: block (b, c), diagonal i; slot s = g bn + j
    // bn, bm and m' are powers of two (zero padding, Sec. 3): shifts and masks
    const int per = a.col_blocks * a.mprime;
    const int b = k / per, c = (k >> a.lmp) % a.col_blocks, i = k & (a.mprime - 1);
    if (a.bsgs > 0) s = (s - (i & -a.bsgs) + a.slots) & (a.slots - 1);  // pre-rotation by the giant step
    const int g = s >> a.lbn, j = s & (a.bn - 1);
    const int rr = (g << a.lmp) + (j & (a.mprime - 1));
    const int row = b * a.bm + rr, col = c * a.bn + ((i + j) & (a.bn - 1));
    return (rr < a.bm && row < a.m && col < a.n) ? (long)row * a.ld + col : -1;
  } else if constexpr (KIND == 1) {  // DIAG: Eq. 5 over max(m,n) slots
    const int row = s & (a.bm - 1), col = (k + s) & (a.bn - 1);
    return (s < a.width && row < a.m && col < a.n) ? (long)row * a.ld + col : -1;
  } else if constexpr (KIND == 2) {  // ROW: row k in slots 0..n-1
    return (s < a.n && k < a.m) ? (long)k * a.ld + s : -1;
  } else if constexpr (KIND == 3) {  // CTMAT: W (n x n_out); plaintext k = i * n_out_cts + kc
    const int i = k / a.n_out_cts, kc = k % a.n_out_cts;
    const int blk = s >> a.lw, j = s & (a.width - 1);
    const int r = (i + j) & (a.bn - 1), col = kc * a.pack + blk;
    return (blk < a.pack && r < a.n && col < a.n_out) ? (long)r * a.ld + col : -1;
  } else {  // COL: plaintext k = j * row_blocks + b holds rows b bm .. of column j
    const int j = k / a.n_out_cts, b = k % a.n_out_cts;
    const int row = b * a.bm + s;
    return (s < a.bm && row < a.m && j < a.n) ? (long)row * a.ld + j : -1;
  }
}

// Element of the encrypted operand that slot t of input ciphertext c holds, or -1.
template <int KIND>
__device__ __forceinline__ long ct_slot_index(const EncodeArgs& a, int c, int t) {
  if constexpr (KIND == 0) {  // HYBRID: column block c of y, period bn
    const int col = c * a.bn + (t & (a.bn - 1));
    return col < a.n ? col : -1;
  } else if constexpr (KIND == 1 || KIND == 2) {  // DIAG / ROW: y with period n_pad
    const int col = t & (a.bn - 1);
    return col < a.n ? col : -1;
  } else if constexpr (KIND == 3) {  // CTMAT: diagonal c of A (m x n), replicated over pack blocks
    const int blk = t >> a.lw, j = t & (a.width - 1);
    const int row = j & (a.bm - 1), col = (c + j) & (a.bn - 1);
    return (blk < a.pack && row < a.m && col < a.n) ? (long)row * a.ld + col : -1;
  } else {  // COL: ciphertext c holds y_c in every slot
    return c < a.n ? (long)c : -1;
  }
}

// v[u] = scale * (value of slot slot_of(u)), u < CNT.  Every load is issued
// before any value is used (a zero slot loads X[0], which exists, and selects
// 0), so the gather pays one memory latency instead of one per slot.
template <bool CT, int KIND, int CNT, class SlotOf>
__device__ __forceinline__ void gather_kind(const EncodeArgs& a, int k, double scale, SlotOf slot_of,
                                            double (&v)[CNT]) {
  long id[CNT];
#pragma unroll
  for (int u = 0; u < CNT; ++u) id[u] = CT ? ct_slot_index<KIND>(a, k, slot_of(u)) : pt_slot_index<KIND>(a, k, slot_of(u));
  double x[CNT];
#pragma unroll
  for (int u = 0; u < CNT; ++u) x[u] = gmem(a.X)[id[u] < 0 ? 0 : id[u]];
#pragma unroll
  for (int u = 0; u < CNT; ++u) v[u] = id[u] < 0 ? 0.0 : x[u] * scale;
}

template <bool CT, int CNT, class SlotOf>
__device__ __forceinline__ void gather_slots(const EncodeArgs& a, int k, double scale, SlotOf slot_of,
                                             double (&v)[CNT]) {
  switch (a.kind) {
    case 0: gather_kind<CT, 0>(a, k, scale, slot_of, v); break;
    case 1: gather_kind<CT, 1>(a, k, scale, slot_of, v); break;
    case 2: gather_kind<CT, 2>(a, k, scale, slot_of, v); break;
    case 3: gather_kind<CT, 3>(a, k, scale, slot_of, v); break;
    default: gather_kind<CT, 4>(a, k, scale, slot_of, v); break;
  }
}

// The slot values v[u] of slots j = tid + u T (u < 8, N <= 2^14) -> FFT ->
// rounded coefficients in registers, as encode_to_regs_v describes.  Slot j
// is DFT input f = (5^j mod 2N - 1) / 4, i.e. component f mod 2 of y[f / 2].
// Begins by writing LDS (barrier before the call if LDS is in use); ends
// with a barrier.
template <int LOGN>
__device__ __forceinline__ void fft_split_regs(const double (&v)[8], double2* z, double* mreg, const EncTabs& et) {
  static_assert(LOGN <= 14, "the 2^15 ring's encoder splits its FFT in halves");
  constexpr int N = 1 << LOGN, M = N / 2, T = NttShape<LOGN>::T, HM = M / 2, QH = HM / T;
  const int tid = opaque_tid();
  const double inv_m = 1.0 / (double)M;
  {
    OrbitWalk ow = OrbitWalk::start<LOGN>();
    double* zd = (double*)z;
#pragma unroll
    for (int u = 0; u < 2 * QH; ++u) {
      const int f = (int)(ow.e >> 2);
      zd[2 * cpad(f >> 1) + (f & 1)] = v[u];
      ow.next<LOGN>();
    }
  }
  __syncthreads();
  fft_passes<LOGN - 1, 0, 1>(z, et.fft_tw, false);
#pragma unroll
  for (int u = 0; u < QH; ++u) {
    const int k = tid + u * T;
    const double2 Yk = z[cpad(brev(k, LOGN - 2))];
    const double2 Yc = z[cpad(brev((HM - k) & (HM - 1), LOGN - 2))];
    const double2 E = make_double2(0.5 * (Yk.x + Yc.x), 0.5 * (Yk.y - Yc.y));
    const double2 O = make_double2(0.5 * (Yk.y + Yc.y), -0.5 * (Yk.x - Yc.x));
    const double2 wo = cmul(O, et.fft_tw[k]);
    const double2 w0 = cmul(make_double2(E.x + wo.x, E.y + wo.y), cconj(et.twist[k]));
    const double2 w1 = cmul(make_double2(E.x - wo.x, E.y - wo.y), cconj(et.twist[k + HM]));
    mreg[2 * u] = round_half_away(w0.x * inv_m);
    mreg[2 * u + 1] = round_half_away(w0.y * inv_m);
    mreg[2 * (u + QH)] = round_half_away(w1.x * inv_m);
    mreg[2 * (u + QH) + 1] = round_half_away(w1.y * inv_m);
  }
  __syncthreads();
}

// slots -> FFT -> rounded coefficients in registers: mreg[2u] = m_k and
// mreg[2u+1] = m_(k+N/2) for k = tid + u T, u < M/T.  gather(slot_of, v)
// fills v[u] with the scaled value of slot slot_of(u) for every u of v.  At N = 2^15 the first DIF stage (pairs i, i + M/2, owned
// by one thread) runs in registers and the two halves in LDS one after the
// other; half h yields the coefficients with k = h mod 2.
template <int LOGN, class Gather>
__device__ __forceinline__ void encode_to_regs_v(Gather gather, double2* z, double* mreg, const EncTabs& et) {
  constexpr int N = 1 << LOGN, M = N / 2, T = NttShape<LOGN>::T;
  const int tid = opaque_tid();
  if constexpr (LOGN <= 14) {
    // The DFT input x[f] (slot value at f = f_j) is real: pack y[n] = x[2n] +
    // i x[2n+1], transform M/2 points, and split (real-input FFT):
    //   E[k] = (Y[k] + conj Y[M/2-k]) / 2,  O[k] = (Y[k] - conj Y[M/2-k]) / 2i,
    //   X[k] = E[k] + W^k O[k],  X[k + M/2] = E[k] - W^k O[k],  W = exp(-2 pi i / M).
    // The half transform runs on the first half of the threads with every
    // other twiddle of the M-point table.
    constexpr int HM = M / 2, QH = HM / T;  // QH = 4 complex inputs per thread
    double v[2 * QH];
    gather([&](int u) { return tid + u * T; }, v);
    fft_split_regs<LOGN>(v, z, mreg, et);
  } else {
    constexpr int HM = M / 2, PH = M / T;
    const double inv_m = 1.0 / (double)M;
    double2 v0[HM / T];
#pragma unroll
    for (int u = 0; u < HM / T; ++u) {
      const int i = tid + u * T;
      double ab[2];
      gather([&](int j) { return (int)et.f2slot[i + j * HM]; }, ab);
      const double a0 = ab[0], b0 = ab[1];
      z[cpad(i)] = make_double2(a0 + b0, 0.0);
      v0[u] = cmul(make_double2(a0 - b0, 0.0), et.fft_tw[i]);
    }
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      if (h) {
        __syncthreads();  // half 0's read-out is done
#pragma unroll
        for (int u = 0; u < HM / T; ++u) z[cpad(tid + u * T)] = v0[u];
      }
      __syncthreads();
      fft_dif_half15(z, et.fft_tw, false);
      if ((tid & 1) == h) {  // k = tid + u T has the parity of tid
#pragma unroll
        for (int u = 0; u < PH; ++u) {
          const int kk = tid + u * T;
          const double2 w = cmul(z[cpad(brev(kk, LOGN - 1) - h * HM)], cconj(et.twist[kk]));
          mreg[2 * u] = round_half_away(w.x * inv_m);
          mreg[2 * u + 1] = round_half_away(w.y * inv_m);
        }
      }
    }
    __syncthreads();
  }
}

template <int LOGN, bool CT>
__device__ __forceinline__ void encode_to_regs(const EncodeArgs& a, int k, double2* z, double* mreg, const EncTabs& et,
                                               double scale) {
  encode_to_regs_v<LOGN>([&](auto slot_of, auto& v) { gather_slots<CT>(a, k, scale, slot_of, v); }, z, mreg, et);
}


// Plaintext k of a plan: pack, encode, then every limb of `map` reduced and
// transformed; written to out_pt[limb][N].  s2: LDS of NttShape<LOGN>::LDS doubles.
template <int LOGN>
__device__ __forceinline__ void encode_pt_body(const EncodeArgs& a, int k, const EncTabs& et, const LimbMap& map,
                                               const DevTabs& tb, double2* s2, double* __restrict__ out_pt) {
  constexpr int N = 1 << LOGN, T = NttShape<LOGN>::T, PH = N / 2 / T, PER = NttShape<LOGN>::PER;
  double* s = (double*)s2;
  double mreg[2 * PH];
  if (a.kind == 2 && k == a.m) {
    // ROW indicator plaintext: 1 in slot 0 at scale q_(l-1)
    const double ind = a.ind_scale;
    encode_to_regs_v<LOGN>(
        [&](auto slot_of, auto& v) {
#pragma unroll
          for (int u = 0; u < (int)(sizeof(v) / sizeof(v[0])); ++u) v[u] = slot_of(u) == 0 ? ind : 0.0;
        },
        s2, mreg, et);
  } else {
    encode_to_regs<LOGN, false>(a, k, s2, mreg, et, a.scale);
  }
  // coefficient tid + w T: w < PH -> m_k (real part), w >= PH -> m_(k+N/2) (imaginary part);
  // |m| < 2^51, which the transform reduces on entry
  for (int l = 0; l < map.n; ++l) {
    const int pi = map.idx[l];
    const ModQ m = tb.mods[pi];
    double c[PER];
#pragma unroll
    for (int w = 0; w < PER; ++w) c[w] = w < PH ? mreg[2 * w] : mreg[2 * (w - PH) + 1];
    // the plaintext buffer is device memory: global stores (unlike flat stores
    // they do not count against the LDS wait counter of the gather before
    // them), nontemporal because nothing in this kernel reads them again --
    // they would only push the twiddle tables and X out of L2
    auto* dst = (__attribute__((address_space(1))) double*)(out_pt + (size_t)l * N);
    ntt_fwd_regs_out<LOGN>(s, c, tb.fwd_tw + (size_t)pi * N, tb.perm, m,
                           [&](int t, double v) { __builtin_nontemporal_store(v, dst + t); });
  }
}

}  // namespace pvfl
