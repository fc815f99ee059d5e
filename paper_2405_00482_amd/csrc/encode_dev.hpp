// Device helpers of the canonical-embedding encoder/decoder and the plan
// packing, shared by the single-plan and the batched kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "encode.hpp"
#include "ntt_core.hpp"

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

// In-place DIF FFT over M = N/2 points in LDS, sign -1 (conj = false) or +1.
template <int LOGN>
__device__ __forceinline__ void fft_dif_lds(double2* a, const double2* __restrict__ tw, bool conj) {
  constexpr int LOGM = LOGN - 1, M = 1 << LOGM;
  constexpr int T = NttShape<LOGN>::T;
  constexpr int BF = M / 2 / T;  // 4
  const int tid = threadIdx.x;
#pragma unroll 1
  for (int s = 0; s < LOGM; ++s) {
    const int lhalf = LOGM - 1 - s;   // log2 of half the current length
    const int half = 1 << lhalf;
#pragma unroll
    for (int r = 0; r < BF; ++r) {
      const int b = tid + r * T;
      const int blk = b >> lhalf, j = b & (half - 1);
      const int i0 = (blk << (lhalf + 1)) + j, i1 = i0 + half;
      double2 w = tw[j << s];  // W_len^j = W_M^(j M/len)
      if (conj) w = cconj(w);
      const double2 u = a[cpad(i0)], v = a[cpad(i1)];
      a[cpad(i0)] = make_double2(u.x + v.x, u.y + v.y);
      a[cpad(i1)] = cmul(make_double2(u.x - v.x, u.y - v.y), w);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int brev(int x, int bits) { return (int)(__brev((unsigned)x) >> (32 - bits)); }

// value of slot s of plaintext k for the plan (0 outside the matrix)
__device__ __forceinline__ double pt_slot_value(const EncodeArgs& a, int k, int s) {
  switch (a.kind) {
    case 0: {  // HYBRID: block (b, c), diagonal i; slot s = g bn + j
      const int per = a.col_blocks * a.mprime;
      const int b = k / per, c = (k / a.mprime) % a.col_blocks, i = k % a.mprime;
      if (a.bsgs > 0) s = (s - (i / a.bsgs) * a.bsgs + a.slots) & (a.slots - 1);  // pre-rotation by the giant step
      const int g = s / a.bn, j = s % a.bn;
      const int rr = g * a.mprime + (j % a.mprime);
      if (rr >= a.bm) return 0.0;
      const int row = b * a.bm + rr, col = c * a.bn + (i + j) % a.bn;
      return (row < a.m && col < a.n) ? a.X[(size_t)row * a.ld + col] : 0.0;
    }
    case 1: {  // DIAG: Eq. 5 over max(m,n) slots
      if (s >= a.width) return 0.0;
      const int row = s % a.bm, col = (k + s) % a.bn;
      return (row < a.m && col < a.n) ? a.X[(size_t)row * a.ld + col] : 0.0;
    }
    case 2: {  // ROW: row k in slots 0..n-1
      return (s < a.n && k < a.m) ? a.X[(size_t)k * a.ld + s] : 0.0;
    }
    case 3: {  // CTMAT: W (n x n_out); plaintext k = i * n_out_cts + kc
      const int i = k / a.n_out_cts, kc = k % a.n_out_cts;
      const int blk = s / a.width, j = s % a.width;
      if (blk >= a.pack) return 0.0;
      const int r = (i + j) % a.bn, col = kc * a.pack + blk;
      return (r < a.n && col < a.n_out) ? a.X[(size_t)r * a.ld + col] : 0.0;
    }
  }
  return 0.0;
}

// value of slot t of input ciphertext c (the encrypted operand)
__device__ __forceinline__ double ct_slot_value(const EncodeArgs& a, int c, int t) {
  switch (a.kind) {
    case 0: {  // HYBRID: column block c of y, period bn
      const int col = c * a.bn + (t % a.bn);
      return col < a.n ? a.X[col] : 0.0;
    }
    case 1:
    case 2: {  // DIAG / ROW: y with period n_pad
      const int col = t % a.bn;
      return col < a.n ? a.X[col] : 0.0;
    }
    case 3: {  // CTMAT: diagonal c of A (m x n), replicated over pack blocks
      const int blk = t / a.width, j = t % a.width;
      if (blk >= a.pack) return 0.0;
      const int row = j % a.bm, col = (c + j) % a.bn;
      return (row < a.m && col < a.n) ? a.X[(size_t)row * a.ld + col] : 0.0;
    }
  }
  return 0.0;
}

// slots -> LDS FFT -> rounded coefficients in registers (mreg[2u] = m_k,
// mreg[2u+1] = m_(k+N/2), k = tid + u T)
template <int LOGN, bool CT>
__device__ __forceinline__ void encode_to_regs(const EncodeArgs& a, int k, double2* z, double* mreg, const EncTabs& et,
                                               double scale) {
  constexpr int N = 1 << LOGN, M = N / 2, T = NttShape<LOGN>::T, PH = M / T;
  const int tid = threadIdx.x;
  for (int s = tid; s < M; s += T) {
    const double v = CT ? ct_slot_value(a, k, s) : pt_slot_value(a, k, s);
    z[cpad(et.slot2f[s])] = make_double2(v * scale, 0.0);
  }
  __syncthreads();
  fft_dif_lds<LOGN>(z, et.fft_tw, false);
  const double inv_m = 1.0 / (double)M;
#pragma unroll
  for (int u = 0; u < PH; ++u) {
    const int kk = tid + u * T;
    const double2 w = cmul(z[cpad(brev(kk, LOGN - 1))], cconj(et.twist[kk]));
    mreg[2 * u] = round_half_away(w.x * inv_m);
    mreg[2 * u + 1] = round_half_away(w.y * inv_m);
  }
  __syncthreads();
}


// Plaintext k of a plan: pack, encode, then every limb of `map` reduced and
// transformed; written to out_pt[limb][N].  s2: LDS of NttShape<LOGN>::LDS doubles.
template <int LOGN>
__device__ __forceinline__ void encode_pt_body(const EncodeArgs& a, int k, const EncTabs& et, const LimbMap& map,
                                               const DevTabs& tb, double2* s2, double* __restrict__ out_pt) {
  constexpr int N = 1 << LOGN, T = NttShape<LOGN>::T, PH = N / 2 / T;
  double* s = (double*)s2;
  double mreg[2 * PH];
  if (a.kind == 2 && k == a.m) {
    // ROW indicator plaintext: 1 in slot 0 at scale q_(l-1)
    for (int t = threadIdx.x; t < N / 2; t += T) s2[cpad(et.slot2f[t])] = make_double2(t == 0 ? a.ind_scale : 0.0, 0.0);
    __syncthreads();
    fft_dif_lds<LOGN>(s2, et.fft_tw, false);
    const double inv_m = 1.0 / (double)(N / 2);
#pragma unroll
    for (int u = 0; u < PH; ++u) {
      const int kk = threadIdx.x + u * T;
      const double2 w = cmul(s2[cpad(brev(kk, LOGN - 1))], cconj(et.twist[kk]));
      mreg[2 * u] = round_half_away(w.x * inv_m);
      mreg[2 * u + 1] = round_half_away(w.y * inv_m);
    }
  } else {
    encode_to_regs<LOGN, false>(a, k, s2, mreg, et, a.scale);
  }
  // coefficient tid + w T: w < 8 -> m_k (real part), w >= 8 -> m_(k+N/2) (imaginary part)
  for (int l = 0; l < map.n; ++l) {
    const int pi = map.idx[l];
    const ModQ m = tb.mods[pi];
    double c[16];
#pragma unroll
    for (int w = 0; w < 16; ++w) c[w] = reduce(w < 8 ? mreg[2 * w] : mreg[2 * (w - 8) + 1], m);
    ntt_fwd_regs<LOGN>(s, c, tb.fwd_tw + (size_t)pi * N, m);
    double* dst = out_pt + (size_t)l * N;
    for (int t = threadIdx.x; t < N; t += T) dst[t] = s[lds_pad(tb.perm[t])];
  }
}

}  // namespace pvfl
