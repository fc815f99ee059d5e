// Negacyclic NTT over binary64-held residues, one ring limb per workgroup,
// the whole limb resident in LDS (N <= 2^14: 128 KiB of the 160 KiB per CU).
//
// Evaluation-domain ("NTT domain") ORDER.  Index t of a transformed limb holds
// a(psi^e(t)) with e(t) = 5^t mod 2N for t < N/2 and e(t) = -5^(t-N/2) mod 2N
// for t >= N/2.  The automorphism X -> X^(5^i) then maps index t to the index
// (t + i) mod N/2 within the same half, so a slot rotation is a cyclic shift of
// contiguous memory instead of a scattered gather.  The butterflies themselves
// run in the textbook bit-reversed order (Cooley-Tukey forward, Gentleman-Sande
// inverse, psi-twist merged into the twiddles); a fixed permutation between
// the bit-reversed index and t is applied when the limb leaves or enters LDS.
//
// Value ranges: inputs may be any integers with |x| < 2^51; butterfly outputs
// are re-centred every few stages so that every mulmod sees |a| <= 4q; outputs
// are centred (|x| <= (q+1)/2).
#pragma once
#include "fp64_mod.hpp"

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
  static constexpr int T = N / 16;        // threads per workgroup
  static constexpr int BF = N / 2 / T;    // butterflies per thread per stage (8)
};

// forward transform of s[0..N) in place: natural coefficient order in,
// bit-reversed evaluation order out (centred).
template <int LOGN>
__device__ __forceinline__ void ntt_fwd_lds(double* s, const double* __restrict__ tw, ModQ m) {
  constexpr int T = NttShape<LOGN>::T;
  constexpr int BF = NttShape<LOGN>::BF;
  const int tid = threadIdx.x;
#pragma unroll 1
  for (int lg = 0; lg < LOGN; ++lg) {
    const int lt = LOGN - 1 - lg;          // log2 of the butterfly span t
    const int t = 1 << lt;
    const bool red = ((lg & 3) == 3) || (lg == LOGN - 1);
#pragma unroll
    for (int r = 0; r < BF; ++r) {
      const int b = tid + r * T;
      const int i = b >> lt;
      const int j = (i << (lt + 1)) + (b & (t - 1));
      const double S = tw[(1 << lg) + i];
      const double U = s[j];
      const double V = mulmod(s[j + t], S, m);
      double x = U + V, y = U - V;
      if (red) { x = reduce(x, m); y = reduce(y, m); }
      s[j] = x;
      s[j + t] = y;
    }
    __syncthreads();
  }
}

// inverse transform in place: bit-reversed evaluation order in, natural
// coefficient order out, scaled by N^-1 and centred.
template <int LOGN>
__device__ __forceinline__ void ntt_inv_lds(double* s, const double* __restrict__ itw, ModQ m, double ninv) {
  constexpr int N = NttShape<LOGN>::N;
  constexpr int T = NttShape<LOGN>::T;
  constexpr int BF = NttShape<LOGN>::BF;
  const int tid = threadIdx.x;
#pragma unroll 1
  for (int lg = LOGN - 1; lg >= 0; --lg) {
    const int lt = LOGN - 1 - lg;
    const int t = 1 << lt;
    const bool red = (lt & 1) == 1;
#pragma unroll
    for (int r = 0; r < BF; ++r) {
      const int b = tid + r * T;
      const int i = b >> lt;
      const int j = (i << (lt + 1)) + (b & (t - 1));
      const double S = itw[(1 << lg) + i];
      const double U = s[j];
      const double V = s[j + t];
      double x = U + V;
      if (red) x = reduce(x, m);
      s[j] = x;
      s[j + t] = mulmod(U - V, S, m);
    }
    __syncthreads();
  }
  for (int k = tid; k < N; k += T) s[k] = reduce(mulmod(s[k], ninv, m), m);
  __syncthreads();
}

}  // namespace pvfl
