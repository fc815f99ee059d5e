// Negacyclic NTT over binary64-held residues, one ring limb per workgroup,
// the whole limb resident in LDS (N <= 2^14: 136 KiB of the 160 KiB per CU).
//
// Evaluation-domain ("NTT domain") ORDER.  Index t of a transformed limb holds
// a(psi^e(t)) with e(t) = 5^t mod 2N for t < N/2 and e(t) = -5^(t-N/2) mod 2N
// for t >= N/2.  The automorphism X -> X^(5^i) then maps index t to the index
// (t + i) mod N/2 within the same half, so a slot rotation is a cyclic shift of
// contiguous memory instead of a scattered gather.  The butterflies run in the
// textbook bit-reversed order (Cooley-Tukey forward, Gentleman-Sande inverse,
// psi-twist merged into the twiddles); a fixed permutation between the
// bit-reversed index and t is applied when the limb leaves or enters LDS.
//
// Schedule.  N/16 threads each hold 16 elements in registers; up to four
// radix-2 stages run on them between two LDS exchanges ("passes"), so a 2^14
// transform makes four LDS round trips instead of fourteen.  In either
// direction only one exchange crosses waves; the other passes stay inside
// one wave's 1024 elements and need no workgroup barrier (see ntt_fwd_regs
// and ntt_inv_regs).  The LDS array is padded by one double every 16 (lds_pad)
// so that the strided set loads of every pass are close to bank-conflict
// free.  The orbit-order permutation is computed from powers of 5 (OrbitWalk)
// rather than read from a table, up to N = 2^14.
//
// Value ranges (q < 2^48): inputs may be any integers with |x| < 2^51.  A
// twiddle mulmod of |a| <= 2^51 by a centred twiddle returns |r| <= 0.875 q
// (its quotient estimate is within 0.875 of the true quotient), so a forward
// butterfly grows values by at most 0.875 q.  Re-centring (to |x| <= q/2) at
// least every 9 stages keeps every butterfly input below q/2 + 8 * 0.875 q =
// 7.5 q < 2^51.  The inverse re-centres its sums every second stage.
// Outputs are centred.
#pragma once
#include "fp64_mod.hpp"

#include <type_traits>

namespace pvfl {

struct DevTabs {
  const ModQ* mods;        // [n_mod]
  const double* fwd_tw;    // [n_mod][N]  psi^brv(k), centred
  const double* inv_tw;    // [n_mod][N]  psi^-brv(k), centred
  const double* ninv;      // [n_mod]     N^-1 mod q, centred
  const double* two32;     // [n_mod]     2^32 mod q, centred
  const uint32_t* perm;    // [N]         orbit index t -> bit-reversed index
  int logN;
};

template <int LOGN>
struct NttShape {
  static constexpr int N = 1 << LOGN;
  // log2 of the transform held in LDS at once: the whole limb up to 2^14; a
  // 2^15 limb (256 KiB) is done as one radix-2 stage plus two 2^14 halves
  static constexpr int LOGH = LOGN < 15 ? LOGN : 14;
  static constexpr int T = (1 << LOGH) / 16;    // threads per workgroup
  static constexpr int PER = N / T;             // coefficients per thread: 16, or 32 at 2^15
  static constexpr int LDS = (1 << LOGH) + (1 << LOGH) / 16;  // padded LDS doubles
};

__device__ __forceinline__ int lds_pad(int j) { return j + (j >> 4); }

// Global-memory views of device pointers.  A load through a generic pointer
// is a flat load, which the hardware counts against the LDS wait counter as
// well: waiting for a kernel's LDS reads would then also wait for every
// global load in flight.  Global loads count against the vector-memory
// counter only.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// The thread index.  A source file that defines PVFL_OPAQUE_TID before
// including this header gets it hidden from loop-invariant code motion (the
// empty asm statement may change it as far as the compiler knows): its
// kernels loop over many limbs, and would otherwise hoist every index and
// address computed from the thread index out of the loop and keep them all
// live in registers at once, which spills.  Elsewhere the compiler keeps
// those values, which saves recomputing them.
static __device__ __forceinline__ int opaque_tid() {
  unsigned t = threadIdx.x;
#if defined(PVFL_OPAQUE_TID)
  asm volatile("" : "+v"(t));
#endif
  return (int)t;
}

// Pass geometry.  A pass of S radix-2 stages works on register sets of 2^S
// elements {base + u * 2^ls} (2^ls = span of the pass's last stage); thread
// tid owns sets c = q*T + tid, q < 16 / 2^S, with base = blk * 2^(ls+S) + off,
// blk = c >> ls, off = c mod 2^ls.  Strides are powers of two, so the index
// arithmetic is shifts and masks.
template <int LOGN, int S>
__device__ __forceinline__ void pass_bases(int (&base)[16 >> S], int ls) {
  constexpr int T = NttShape<LOGN>::T;
#pragma unroll
  for (int q = 0; q < (16 >> S); ++q) {
    const unsigned c = (unsigned)(q * T) + opaque_tid();
    base[q] = (int)(((c >> ls) << (ls + S)) | (c & ((1u << ls) - 1u)));
  }
}

// S radix-2 Cooley-Tukey stages lg0 .. lg0+S-1 on the register sets.  A set
// lies inside one butterfly group of stage lg0 (group g0 = base >> (LOGN -
// lg0)); at stage lg0 + st it spans 2^st groups g0 * 2^st + k, whose
// twiddles are contiguous in the table, so a pass reads 2^S - 1 twiddles per
// set.  No reduction here: a butterfly adds less than q in magnitude (the
// mulmod output is below q), and the caller re-centres often enough that
// every value stays below 2^51.
template <int LOGN, int S>
__device__ __forceinline__ void ct_pass_regs(double (&x)[16], int lg0, const int (&base)[16 >> S],
                                             const double* __restrict__ tw, ModQ m) {
  constexpr int SET = 1 << S;
#pragma unroll
  for (int q = 0; q < (16 >> S); ++q) {
    const int g0 = base[q] >> (LOGN - lg0);
#pragma unroll
    for (int st = 0; st < S; ++st) {
      const int half = SET >> (st + 1);
      double w[1 << (S > 0 ? S - 1 : 0)];
      const double* tws = tw + (1 << (lg0 + st)) + (g0 << st);
#pragma unroll
      for (int k = 0; k < (1 << st); ++k) w[k] = tws[k];
#pragma unroll
      for (int u = 0; u < SET; ++u) {
        if (u & half) continue;
        const double U = x[q * SET + u];
        const double V = mulmod(x[q * SET + u + half], w[u >> (S - st)], m);
        x[q * SET + u] = U + V;
        x[q * SET + u + half] = U - V;
      }
    }
  }
}

template <int N>
__device__ __forceinline__ void recentre(double (&x)[N], ModQ m) {
#pragma unroll
  for (int k = 0; k < N; ++k) x[k] = reduce(x[k], m);
}

// Sets with a compile-time span 2^LS: element u of a set lies at padded
// offset (u << LS) + ((u << LS) >> 4) from the set's base.  This holds when
// the base is below 2^LS modulo 2^(LS+4) (then adding u 2^LS never carries
// into a new run of 16 except through the multiple-of-16 part), which every
// pass of the forward transform guarantees.
template <int S, int LS, int NQ>
__device__ __forceinline__ void lds_load_c(const double* s, double (&x)[16], const int (&base)[NQ]) {
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double* p = s + lds_pad(base[q]);
#pragma unroll
    for (int u = 0; u < (1 << S); ++u) x[q * (1 << S) + u] = p[(u << LS) + ((u << LS) >> 4)];
  }
}
template <int S, int LS, int NQ>
__device__ __forceinline__ void lds_store_c(double* s, const double (&x)[16], const int (&base)[NQ]) {
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double* p = s + lds_pad(base[q]);
#pragma unroll
    for (int u = 0; u < (1 << S); ++u) p[(u << LS) + ((u << LS) >> 4)] = x[q * (1 << S) + u];
  }
}

// Orders a wave's LDS stores before its later LDS loads of what other lanes
// of the same wave stored (LDS operations of one wave execute in order; the
// fences keep the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Forward transform (2^12 <= N <= 2^14, N/16 threads).  c[w] is coefficient
// tid + w*T of the thread (natural order, any |x| < 2^51).  Schedule:
//  * stages 0..3 (spans N/2 .. N/16) on the thread's own 16 coefficients,
//    which form one radix-16 set, in registers;
//  * one exchange through LDS behind a workgroup barrier, after which wave
//    w owns the 1024 consecutive elements [1024 w, 1024 w + 1024);
//  * stages 4..7 and 8..11 as radix-16 sets, and the last LOGN - 12 stages
//    as sets of consecutive elements, all inside the wave's own 1024
//    elements: these exchanges go through the wave's part of LDS with no
//    workgroup barrier, so the waves drift apart and one wave's LDS traffic
//    overlaps another's arithmetic.
// Re-centring after stage 7 and at the end (at most 8 stages between two).
// The result is left in LDS in bit-reversed order, centred: read it with
// s[lds_pad(j)] after the call (which ends with a barrier).  The call begins
// with a barrier, so `s` may still be in use by the caller before it.
template <int LOGN>
__device__ __forceinline__ void ntt_fwd_regs(double* s, const double (&c)[16], const double* __restrict__ tw, ModQ m) {
  static_assert(LOGN >= 12 && LOGN <= 14, "one wave owns 1024 elements of an LDS-resident limb");
  double x[16];
  const int tid = opaque_tid();
  // the first stage adds x[u] (u < 8) to a twiddle product of x[u + 8]:
  // mulmod takes |x[u + 8]| < 2^51 as it is, so only the addends are
  // re-centred, and every value after the stage obeys the same bound
#pragma unroll
  for (int u = 0; u < 8; ++u) x[u] = reduce(c[u], m);
#pragma unroll
  for (int u = 8; u < 16; ++u) x[u] = c[u];
  {
    const int base[1] = {tid};
    ct_pass_regs<LOGN, 4>(x, 0, base, tw, m);
    __syncthreads();
    lds_store_c<4, LOGN - 4>(s, x, base);
  }
  __syncthreads();
  {  // stages 4..7: sets {base + u 2^(LOGN-8)} inside the wave's 1024 elements
    constexpr int LS = LOGN - 8;
    int base[1];
    pass_bases<LOGN, 4>(base, LS);
    lds_load_c<4, LS>(s, x, base);
    ct_pass_regs<LOGN, 4>(x, 4, base, tw, m);
    recentre(x, m);
    lds_store_c<4, LS>(s, x, base);
  }
  wave_lds_sync();
  {  // stages 8..11
    constexpr int LS = LOGN - 12;
    int base[1];
    pass_bases<LOGN, 4>(base, LS);
    lds_load_c<4, LS>(s, x, base);
    ct_pass_regs<LOGN, 4>(x, 8, base, tw, m);
    if constexpr (LOGN == 12) recentre(x, m);
    lds_store_c<4, LS>(s, x, base);
  }
  if constexpr (LOGN > 12) {  // stages 12 .. LOGN-1: sets of 2^S consecutive elements, 16 per thread
    constexpr int S = LOGN - 12, NQ = 16 >> S;
    wave_lds_sync();
    int base[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) base[q] = 16 * tid + (q << S);
    lds_load_c<S, 0>(s, x, base);
    ct_pass_regs<LOGN, S>(x, 12, base, tw, m);
    recentre(x, m);
    lds_store_c<S, 0>(s, x, base);
  }
  __syncthreads();
}

// forward transform of coefficients produced by load(j)
template <int LOGN, class Load>
__device__ __forceinline__ void ntt_fwd(double* s, Load load, const double* __restrict__ tw, ModQ m) {
  constexpr int T = NttShape<LOGN>::T;
  double c[16];
#pragma unroll
  for (int w = 0; w < 16; ++w) c[w] = load((int)opaque_tid() + w * T);
  ntt_fwd_regs<LOGN>(s, c, tw, m);
}

// S Gentleman-Sande stages lg1, lg1-1, ..., lg1-S+1 (span doubling each
// stage); sets {base + u * 2^ls}, 2^ls = span of the first stage.  The set is
// one group of stage lg1-S+1; at stage lg1-st it spans 2^(S-1-st) groups with
// contiguous twiddles.  Sums are re-centred every second stage, differences
// go through mulmod; everything is re-centred at the end.
template <int LOGN, int S>
__device__ __forceinline__ void gs_pass_regs(double (&x)[16], int lg1, const int (&base)[16 >> S],
                                             const double* __restrict__ itw, ModQ m) {
  constexpr int SET = 1 << S;
#pragma unroll
  for (int q = 0; q < (16 >> S); ++q) {
#pragma unroll
    for (int st = 0; st < S; ++st) {
      const int lg = lg1 - st;
      const int half = 1 << st;
      const int gbase = base[q] >> (LOGN - lg);  // group of element u = 0 at this stage
      double w[1 << (S > 0 ? S - 1 : 0)];
      const double* tws = itw + (1 << lg) + gbase;
#pragma unroll
      for (int k = 0; k < (SET >> (st + 1)); ++k) w[k] = tws[k];
#pragma unroll
      for (int u = 0; u < SET; ++u) {
        if (u & half) continue;
        const double U = x[q * SET + u];
        const double V = x[q * SET + u + half];
        double sum = U + V;
        if (st & 1) sum = reduce(sum, m);
        x[q * SET + u] = sum;
        x[q * SET + u + half] = mulmod(U - V, w[u >> (st + 1)], m);
      }
    }
  }
  recentre(x, m);
}

// Inverse transform of the bit-reversed data already in LDS (padded, after a
// barrier).  On return c[w] is coefficient tid + w*T of the natural-order
// result times N^-1, centred.  LDS is still being read by other threads when
// this returns: barrier before writing `s` again (ntt_fwd_regs does).
// Schedule (the forward one mirrored): the first LOGN - 4 stages (spans 1
// .. N/32) stay inside wave w's 1024 elements [1024 w, 1024 w + 1024) --
// LOGN - 12 stages on sets of consecutive elements, then two radix-16
// passes -- with wave-local LDS exchanges; after one workgroup barrier the
// last four stages (spans N/16 .. N/2) run on the thread's own coefficients
// {tid + u N/16}.
template <int LOGN>
__device__ __forceinline__ void ntt_inv_regs(double* s, double (&c)[16], const double* __restrict__ itw, ModQ m,
                                             double ninv) {
  static_assert(LOGN >= 12 && LOGN <= 14, "one wave owns 1024 elements of an LDS-resident limb");
  double x[16];
  const int tid = opaque_tid();
  if constexpr (LOGN > 12) {  // stages of span 1 .. 2^(S-1): sets of 2^S consecutive elements
    constexpr int S = LOGN - 12, NQ = 16 >> S;
    int base[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) base[q] = 16 * tid + (q << S);
    lds_load_c<S, 0>(s, x, base);
    gs_pass_regs<LOGN, S>(x, LOGN - 1, base, itw, m);
    lds_store_c<S, 0>(s, x, base);
    wave_lds_sync();
  }
  {  // four stages from span 2^(LOGN-12)
    constexpr int LS = LOGN - 12;
    int base[1];
    pass_bases<LOGN, 4>(base, LS);
    lds_load_c<4, LS>(s, x, base);
    gs_pass_regs<LOGN, 4>(x, 11, base, itw, m);
    lds_store_c<4, LS>(s, x, base);
  }
  wave_lds_sync();
  {  // four stages from span 2^(LOGN-8)
    constexpr int LS = LOGN - 8;
    int base[1];
    pass_bases<LOGN, 4>(base, LS);
    lds_load_c<4, LS>(s, x, base);
    gs_pass_regs<LOGN, 4>(x, 7, base, itw, m);
    lds_store_c<4, LS>(s, x, base);
  }
  __syncthreads();
  {  // spans N/16 .. N/2 on the thread's coefficients tid + u N/16
    const int base[1] = {tid};
    lds_load_c<4, LOGN - 4>(s, x, base);
    gs_pass_regs<LOGN, 4>(x, 3, base, itw, m);
#pragma unroll
    for (int u = 0; u < 16; ++u) c[u] = reduce(mulmod(x[u], ninv, m), m);
  }
}

// inverse transform handing coefficient j to store(j, v)
template <int LOGN, class Store>
__device__ __forceinline__ void ntt_inv(double* s, Store store, const double* __restrict__ itw, ModQ m, double ninv) {
  constexpr int T = NttShape<LOGN>::T;
  double c[16];
  ntt_inv_regs<LOGN>(s, c, itw, m, ninv);
#pragma unroll
  for (int w = 0; w < 16; ++w) store((int)opaque_tid() + w * T, c[w]);
}


// Orbit order <-> bit-reversed index, computed instead of read from the
// table (2^12 <= N <= 2^14).  Slot t < N/2 holds the exponent e = 5^t mod 2N,
// at bit-reversed index brv((e - 1) / 2); slot t + N/2 holds -e, at the
// complement (N - 1) - brv((e - 1) / 2).  A thread's slots t = tid + w N/16
// have e = 5^tid (5^(N/16))^w: as 2N is a power of two every product is
// exact in 32 bits and the reduction is a mask.
template <int LOGN>
constexpr uint32_t pow5_step() {  // 5^(N/16) mod 2N
  uint32_t r = 1;
  for (int i = 0; i < (1 << LOGN) / 16; ++i) r = (r * 5u) & ((2u << LOGN) - 1u);
  return r;
}
struct OrbitWalk {
  uint32_t e;  // 5^(tid + w N/16) mod 2N for the thread's current w
  template <int LOGN>
  __device__ __forceinline__ static OrbitWalk start() {  // 5^tid mod 2N, tid < N/16
    const uint32_t mask = (2u << LOGN) - 1u, tid = opaque_tid();
    uint32_t r = 1, b = 5;
#pragma unroll
    for (int k = 0; k < LOGN - 4; ++k) {
      if ((tid >> k) & 1u) r = (r * b) & mask;
      b = (b * b) & mask;
    }
    return OrbitWalk{r};
  }
  template <int LOGN>
  __device__ __forceinline__ int brv_index() const { return (int)(__brev(e >> 1) >> (32 - LOGN)); }
  template <int LOGN>
  __device__ __forceinline__ void next() {
    e = (e * std::integral_constant<uint32_t, pow5_step<LOGN>()>::value) & ((2u << LOGN) - 1u);
  }
};

// ---------------------------------------------------------------------------
// Size-generic entry points.  Thread tid owns coefficients j = tid + w*T,
// w < PER, and the evaluation-domain (orbit-order) slots t = tid + u*T.
//
// At N = 2^15 the limb does not fit in LDS.  The forward transform's first
// Cooley-Tukey stage pairs j and j + N/2, which the same thread owns (w and
// w + 16), so it runs in registers; the two halves are then independent 2^14
// transforms whose twiddles are the full table's entries re-indexed per half
// (the host stores half h's table at offset h * 2^14 of the prime's row and
// the first stage's twiddle at index 0, unused by the 2^14 transform).  The
// bit-reversed half h holds exactly the orbit slots [h N/2, (h+1) N/2) (odd
// exponents 5^t are 1 mod 4, -5^t are 3 mod 4), so each half is written out
// contiguously.  The inverse runs the two halves' Gentleman-Sande stages in
// LDS one after the other and their last stage (span N/2) in registers.
// ---------------------------------------------------------------------------
template <int LOGN, class Out>
__device__ __forceinline__ void ntt_fwd_regs_out(double* s, const double (&c)[NttShape<LOGN>::PER],
                                                 const double* __restrict__ tw, const uint32_t* __restrict__ perm,
                                                 ModQ m, Out out) {
  constexpr int N = 1 << LOGN, T = NttShape<LOGN>::T;
  if constexpr (LOGN <= 14) {
    ntt_fwd_regs<LOGN>(s, c, tw, m);
    // slots t and t + N/2 for two w at a time: four LDS reads in flight
    OrbitWalk ow = OrbitWalk::start<LOGN>();
#pragma unroll 1
    for (int w = 0; w < 8; w += 2) {
      int j[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        j[h] = ow.brv_index<LOGN>();
        ow.next<LOGN>();
      }
      double v[4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        v[2 * h] = s[lds_pad(j[h])];
        v[2 * h + 1] = s[lds_pad(j[h] ^ (N - 1))];
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        out((int)opaque_tid() + (w + h) * T, v[2 * h]);
        out((int)opaque_tid() + (w + h) * T + N / 2, v[2 * h + 1]);
      }
    }
  } else {
    constexpr int H = 1 << 14;
    const double w0 = tw[0];
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      double x[16];
#pragma unroll
      for (int w = 0; w < 16; ++w) {
        const double U = reduce(c[w], m), V = mulmod(c[w + 16], w0, m);
        x[w] = h ? U - V : U + V;
      }
      ntt_fwd_regs<14>(s, x, tw + h * H, m);
      for (int t = h * (N / 2) + (int)opaque_tid(); t < (h + 1) * (N / 2); t += T) out(t, s[lds_pad(perm[t] - h * H)]);
    }
  }
}

// forward transform of the coefficients load(j), handing slot t to out(t, v)
template <int LOGN, class Load, class Out>
__device__ __forceinline__ void ntt_fwd_out(double* s, Load load, const double* __restrict__ tw,
                                            const uint32_t* __restrict__ perm, ModQ m, Out out) {
  constexpr int T = NttShape<LOGN>::T, PER = NttShape<LOGN>::PER;
  double c[PER];
#pragma unroll
  for (int w = 0; w < PER; ++w) c[w] = load((int)opaque_tid() + w * T);
  ntt_fwd_regs_out<LOGN>(s, c, tw, perm, m, out);
}

// Inverse transform of the orbit-order values in(t) (|x| < 2^51); c[w] gets
// coefficient tid + w*T times N^-1, centred.  LDS may still be read by other
// threads on return: barrier before writing `s` again.
template <int LOGN, class In>
__device__ __forceinline__ void ntt_inv_in_regs(double* s, In in, const double* __restrict__ itw,
                                                const uint32_t* __restrict__ perm, ModQ m, double ninv,
                                                double (&c)[NttShape<LOGN>::PER]) {
  constexpr int N = 1 << LOGN, T = NttShape<LOGN>::T;
  if constexpr (LOGN <= 14) {
    OrbitWalk ow = OrbitWalk::start<LOGN>();
#pragma unroll 2
    for (int w = 0; w < 8; ++w) {
      const int t = (int)opaque_tid() + w * T, j = ow.brv_index<LOGN>();
      s[lds_pad(j)] = reduce(in(t), m);
      s[lds_pad(j ^ (N - 1))] = reduce(in(t + N / 2), m);
      ow.next<LOGN>();
    }
    __syncthreads();
    ntt_inv_regs<LOGN>(s, c, itw, m, ninv);
  } else {
    constexpr int H = 1 << 14;
    double c0[16], c1[16];
    for (int t = opaque_tid(); t < N / 2; t += T) s[lds_pad(perm[t])] = reduce(in(t), m);
    __syncthreads();
    ntt_inv_regs<14>(s, c0, itw, m, ninv);
    __syncthreads();
    for (int t = N / 2 + (int)opaque_tid(); t < N; t += T) s[lds_pad(perm[t] - H)] = reduce(in(t), m);
    __syncthreads();
    ntt_inv_regs<14>(s, c1, itw + H, m, ninv);
    const double iw0 = itw[0];
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      c[w] = reduce(c0[w] + c1[w], m);
      c[w + 16] = reduce(mulmod(c0[w] - c1[w], iw0, m), m);
    }
  }
}

// inverse transform of in(t), handing coefficient j to store(j, v)
template <int LOGN, class In, class Store>
__device__ __forceinline__ void ntt_inv_in(double* s, In in, const double* __restrict__ itw,
                                           const uint32_t* __restrict__ perm, ModQ m, double ninv, Store store) {
  constexpr int T = NttShape<LOGN>::T, PER = NttShape<LOGN>::PER;
  double c[PER];
  ntt_inv_in_regs<LOGN>(s, in, itw, perm, m, ninv, c);
#pragma unroll
  for (int w = 0; w < PER; ++w) store((int)opaque_tid() + w * T, c[w]);
}

}  // namespace pvfl
