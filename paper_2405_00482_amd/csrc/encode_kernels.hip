// Canonical-embedding encode/decode (FP64, gfx950) and the plaintext packing
// of the plans.
//
// Slots z_j (j < N/2) are the values at zeta^(5^j), zeta = exp(i pi / N).  With
// e_j = 5^j mod 2N = 4 f_j + 1 and w_k = m_k + i m_(k+N/2) (k < N/2):
//     z_j = sum_k (w_k zeta^k) W^(-k f_j),   W = exp(-2 pi i / (N/2)),
// a length-N/2 DFT of the twisted w, read at index f_j.  Encoding inverts it:
// place scale*z_j at f_j, forward DFT / (N/2), untwist by zeta^-k, round the
// real and imaginary parts half away from zero to m_k and m_(k+N/2).
// The complex transform runs in LDS (N/2 complex doubles = 8N bytes) as a
// radix-2 decimation-in-frequency FFT (natural order in, bit-reversed out).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "encode_dev.hpp"

namespace pvfl {

// One workgroup per plaintext: pack, encode, then every limb reduced and
// transformed.  out[k][limb][N].
template <int LOGN>
__global__ __launch_bounds__(NttShape<LOGN>::T) void k_encode_pt(EncodeArgs a, EncTabs et, LimbMap map, DevTabs tb,
                                                                 double* __restrict__ out) {
  __shared__ double2 s2[NttShape<LOGN>::LDS / 2];
  encode_pt_body<LOGN>(a, (int)blockIdx.x, et, map, tb, s2, out + (size_t)blockIdx.x * map.n * (1 << LOGN));
}

// Input ciphertext messages: one workgroup per ciphertext, int64 coefficients
template <int LOGN>
__global__ __launch_bounds__(NttShape<LOGN>::T) void k_encode_ct_msg(EncodeArgs a, EncTabs et, int64_t* __restrict__ msg) {
  constexpr int N = 1 << LOGN, T = NttShape<LOGN>::T, PH = N / 2 / T;
  __shared__ double2 s2[NttShape<LOGN>::LDS / 2];
  const int c = blockIdx.x;
  double mreg[2 * PH];
  encode_to_regs<LOGN, true>(a, c, s2, mreg, et, a.scale);
  int64_t* dst = msg + (size_t)c * N;
#pragma unroll
  for (int u = 0; u < PH; ++u) {
    const int kk = threadIdx.x + u * T;
    dst[kk] = (int64_t)mreg[2 * u];
    dst[kk + N / 2] = (int64_t)mreg[2 * u + 1];
  }
}

// Decode: centred CRT lift of decrypted coefficient residues [nct][l+1][N]
// (canonical, binary64), twist, DFT with sign +1, slots z[c][j] =
// Re(.)/scale.
template <int LOGN>
__global__ __launch_bounds__(NttShape<LOGN>::T) void k_decode(const double* __restrict__ res, int lv, CrtTabs ct,
                                                              EncTabs et, double inv_scale, double* __restrict__ z) {
  constexpr int N = 1 << LOGN, M = N / 2, T = NttShape<LOGN>::T;
  __shared__ double2 w[NttShape<LOGN>::LDS / 2];
  const int c = blockIdx.x;
  const double* base = res + (size_t)c * (lv + 1) * N;
  const int nl = lv + 1;
  auto lift = [&](int kk) { return crt_lift<0>(base, kk, N, ct, nl); };
  // twisted w_k = (m_k + i m_(k+N/2)) zeta^k
  auto twisted = [&](int k) { return cmul(make_double2(lift(k), lift(k + M)), et.twist[k]); };
  double* zc = z + (size_t)c * M;
  if constexpr (LOGN <= 14) {
    decode_to_lds<LOGN>(base, nl, ct, et, w);
    for (int j = threadIdx.x; j < M; j += T) zc[j] = decoded_slot<LOGN>(w, et, j, inv_scale);
  } else {
    // first DIF stage (pairs k, k + M/2) in registers, then the two halves in LDS
    constexpr int HM = M / 2;
    double2 v0[HM / T];
#pragma unroll
    for (int u = 0; u < HM / T; ++u) {
      const int k = threadIdx.x + u * T;
      const double2 a0 = twisted(k), b0 = twisted(k + HM);
      w[cpad(k)] = make_double2(a0.x + b0.x, a0.y + b0.y);
      v0[u] = cmul(make_double2(a0.x - b0.x, a0.y - b0.y), cconj(et.fft_tw[k]));
    }
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      if (h) {
        __syncthreads();  // half 0's read-out is done
#pragma unroll
        for (int u = 0; u < HM / T; ++u) w[cpad(threadIdx.x + u * T)] = v0[u];
      }
      __syncthreads();
      fft_dif_half15(w, et.fft_tw, true);
      for (int j = threadIdx.x; j < M; j += T) {
        const int r = brev(et.slot2f[j], LOGN - 1);
        if ((r >> (LOGN - 2)) == h) zc[j] = w[cpad(r - h * HM)].x * inv_scale;
      }
    }
  }
}

// Value of slot s of output ciphertext b for a cleartext added to the plan's
// result (mode 0: the m outputs spread by the cleartext inverse RaS of Sec.
// 5.2, each split into equal parts over the slots its row's lazy RaS adds;
// mode 1: slot values [ct_out][N/2] as given).  The parts are powers-of-two
// fractions of v, so the split is exact.
__device__ __forceinline__ double out_slot_value(const EncodeArgs& a, const double* __restrict__ v, int mode,
                                                 int ras_in_ct, int b, int s) {
  if (mode == 1) return v[(size_t)b * a.slots + s];
  switch (a.kind) {
    case 0: {  // HYBRID: slot g bn + j adds into row g m' + (j mod m') of block b
      const int g = s >> a.lbn, j = s & (a.bn - 1);
      const int row = b * a.bm + (g << a.lmp) + (j & (a.mprime - 1));
      return row < a.m ? ldexp(v[row], a.lmp - a.lbn) : 0.0;
    }
    case 1: {  // DIAG over max(m,n) slots
      if (a.bm >= a.bn || ras_in_ct) return s < a.m ? v[s] : 0.0;
      const int r = s & (a.bm - 1);
      return (s < a.bn && r < a.m) ? ldexp(v[r], __builtin_ctz(a.bm) - a.lbn) : 0.0;
    }
    case 4: {  // COL: slot s of output ciphertext b is row b bm + s
      const int row = b * a.bm + s;
      return (s < a.bm && row < a.m) ? v[row] : 0.0;
    }
    case 3: {  // CTMAT: output ciphertext b, column block blk = s / width
      const int blk = s >> a.lw, j = s & (a.width - 1), col = b * a.pack + blk;
      if (blk >= a.pack || col >= a.n_out) return 0.0;
      if (a.bm >= a.bn) return j < a.m ? v[(size_t)j * a.n_out + col] : 0.0;
      const int r = j & (a.bm - 1);
      return (j < a.bn && r < a.m) ? ldexp(v[(size_t)r * a.n_out + col], __builtin_ctz(a.bm) - a.lbn) : 0.0;
    }
  }
  return 0.0;
}

// One workgroup per output ciphertext: the cleartext at scale a.scale,
// rounded, then every limb's residues times fac[l] (2^e mod q) and transformed.
template <int LOGN>
__global__ __launch_bounds__(NttShape<LOGN>::T) void k_encode_out(EncodeArgs a, const double* __restrict__ v, int mode,
                                                                  int ras_in_ct, OutFactors fac, EncTabs et, LimbMap map,
                                                                  DevTabs tb, double* __restrict__ out) {
  constexpr int N = 1 << LOGN, T = NttShape<LOGN>::T, PH = N / 2 / T, PER = NttShape<LOGN>::PER;
  __shared__ double2 s2[NttShape<LOGN>::LDS / 2];
  const int b = blockIdx.x;
  double mreg[2 * PH];
  encode_to_regs_v<LOGN>(
      [&](auto slot_of, auto& val) {
#pragma unroll
        for (int u = 0; u < (int)(sizeof(val) / sizeof(val[0])); ++u)
          val[u] = out_slot_value(a, v, mode, ras_in_ct, b, slot_of(u)) * a.scale;
      },
      s2, mreg, et);
  double* s = (double*)s2;
  for (int l = 0; l < map.n; ++l) {
    const ModQ m = tb.mods[map.idx[l]];
    double c[PER];
#pragma unroll
    for (int w = 0; w < PER; ++w) c[w] = mulmod(w < PH ? mreg[2 * w] : mreg[2 * (w - PH) + 1], fac.f[l], m);
    double* dst = out + ((size_t)b * map.n + l) * N;
    ntt_fwd_regs_out<LOGN>(s, c, tb.fwd_tw + (size_t)map.idx[l] * N, tb.perm, m, [&](int t, double x) { dst[t] = x; });
  }
}

// out c0 = ct c0 + sign * pt, c1 copied, on nct ciphertexts of lv+1 limbs
__global__ __launch_bounds__(256) void k_out_add_pt(const double* __restrict__ ct, const double* __restrict__ pt, double sign,
                                                    int nct, int lv, int N, const ModQ* __restrict__ mods,
                                                    double* __restrict__ out) {
  const size_t Q = (size_t)(lv + 1) * N;
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)nct * 2 * Q) return;
  const size_t c = idx / (2 * Q), r = idx % (2 * Q);
  if (r >= Q) {
    out[idx] = ct[idx];
    return;
  }
  const int i = (int)(r / N);
  out[idx] = reduce(ct[idx] + sign * pt[c * Q + r], mods[i]);
}

// lazy rotate-and-sum / read-out of the decoded slots (Sec. 4.3)
__global__ __launch_bounds__(256) void k_readout(const double* __restrict__ z, EncodeArgs a, int ras_in_ct,
                                                 double* __restrict__ y) {
  const int M = a.slots;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  switch (a.kind) {
    case 0: {
      if (idx >= a.m) return;
      const int b = idx / a.bm, rr = idx % a.bm, g = rr / a.mprime, rho = rr % a.mprime;
      const double* zb = z + (size_t)b * M;
      double acc = 0.0;
      for (int t = 0; t < a.bn / a.mprime; ++t) acc += zb[g * a.bn + rho + t * a.mprime];
      y[idx] = acc;
      return;
    }
    case 1: {
      if (idx >= a.m) return;
      if (a.bm >= a.bn || ras_in_ct) { y[idx] = z[idx]; return; }
      double acc = 0.0;
      for (int t = 0; t < a.bn / a.bm; ++t) acc += z[idx + t * a.bm];
      y[idx] = acc;
      return;
    }
    case 2:
      if (idx < a.m) y[idx] = z[idx];
      return;
    case 4:  // COL: row block b of N/2 rows, no rotate-and-sum
      if (idx < a.m) y[idx] = z[(size_t)(idx / a.bm) * M + idx % a.bm];
      return;
    case 3: {
      if (idx >= a.m * a.n_out) return;
      const int r = idx / a.n_out, col = idx % a.n_out;
      const int kc = col / a.pack, blk = col % a.pack;
      const double* zk = z + (size_t)kc * M + (size_t)blk * a.width;
      if (a.bm >= a.bn) { y[idx] = zk[r]; return; }
      double acc = 0.0;
      for (int t = 0; t < a.bn / a.bm; ++t) acc += zk[r + t * a.bm];
      y[idx] = acc;
      return;
    }
  }
}

// ---------------------------------------------------------------------------
template <int LOGN>
static void encode_pt_impl(const LaunchCtx& L, const EncodeArgs& a, const EncTabs& et, LimbMap map, int count, double* out) {
  hipLaunchKernelGGL(k_encode_pt<LOGN>, dim3(count), dim3(NttShape<LOGN>::T), 0, L.stream, a, et, map, L.tb, out);
}
template <int LOGN>
static void encode_out_impl(const LaunchCtx& L, const EncodeArgs& a, const double* v, int mode, int ras_in_ct,
                            const OutFactors& fac, const EncTabs& et, LimbMap map, int count, double* out) {
  hipLaunchKernelGGL(k_encode_out<LOGN>, dim3(count), dim3(NttShape<LOGN>::T), 0, L.stream, a, v, mode, ras_in_ct, fac,
                     et, map, L.tb, out);
}
template <int LOGN>
static void encode_ct_impl(const LaunchCtx& L, const EncodeArgs& a, const EncTabs& et, int count, int64_t* msg) {
  hipLaunchKernelGGL(k_encode_ct_msg<LOGN>, dim3(count), dim3(NttShape<LOGN>::T), 0, L.stream, a, et, msg);
}
template <int LOGN>
static void decode_impl(const LaunchCtx& L, const double* res, int nct, int lv, const CrtTabs& ct, const EncTabs& et,
                        double inv_scale, double* z) {
  hipLaunchKernelGGL(k_decode<LOGN>, dim3(nct), dim3(NttShape<LOGN>::T), 0, L.stream, res, lv, ct, et, inv_scale, z);
}

#define DISPATCH_LOGN(L, FN, ...)                         \
  switch ((L).logN) {                                     \
    case 12: FN<12>(__VA_ARGS__); break;                  \
    case 13: FN<13>(__VA_ARGS__); break;                  \
    case 14: FN<14>(__VA_ARGS__); break;                  \
    case 15: FN<15>(__VA_ARGS__); break;                  \
    default: return hipErrorInvalidValue;                 \
  }

hipError_t launch_encode_pt(const LaunchCtx& L, const EncodeArgs& a, const EncTabs& et, LimbMap map, int count,
                            double* out) {
  if (count <= 0) return hipSuccess;
  DISPATCH_LOGN(L, encode_pt_impl, L, a, et, map, count, out);
  return hipGetLastError();
}
hipError_t launch_encode_ct(const LaunchCtx& L, const EncodeArgs& a, const EncTabs& et, int count, int64_t* msg) {
  DISPATCH_LOGN(L, encode_ct_impl, L, a, et, count, msg);
  return hipGetLastError();
}
hipError_t launch_decode(const LaunchCtx& L, const double* res, int nct, int lv, const CrtTabs& ct, const EncTabs& et,
                         double inv_scale, double* z) {
  DISPATCH_LOGN(L, decode_impl, L, res, nct, lv, ct, et, inv_scale, z);
  return hipGetLastError();
}
hipError_t launch_encode_out(const LaunchCtx& L, const EncodeArgs& a, const double* v, int mode, int ras_in_ct,
                             const OutFactors& fac, const EncTabs& et, LimbMap map, int count, double* out) {
  if (count <= 0) return hipSuccess;
  DISPATCH_LOGN(L, encode_out_impl, L, a, v, mode, ras_in_ct, fac, et, map, count, out);
  return hipGetLastError();
}
hipError_t launch_out_add_pt(const LaunchCtx& L, const double* ct, const double* pt, double sign, int nct, int lv, int N,
                             double* out) {
  const size_t tot = (size_t)nct * 2 * (lv + 1) * N;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_out_add_pt, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, L.stream, ct, pt, sign, nct, lv, N,
                     L.tb.mods, out);
  return hipGetLastError();
}
hipError_t launch_readout(const LaunchCtx& L, const double* z, const EncodeArgs& a, int ras_in_ct, int count, double* y) {
  hipLaunchKernelGGL(k_readout, dim3((count + 255) / 256), dim3(256), 0, L.stream, z, a, ras_in_ct, y);
  return hipGetLastError();
}

}  // namespace pvfl
