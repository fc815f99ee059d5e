// Batched execution of many independent products (uneven shapes) sharing one
// context, level and rotation-key set: every phase of the path is one launch
// over all products, and the fused diagonal kernel streams each rotation key
// once per group of products instead of once per product.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch.hpp"
#include "encode_dev.hpp"
#include "he_dev.hpp"

namespace pvfl {

// ---------------------------------------------------------------------------
// fused hoisted rotations x diagonals, lazy ModDown, shared keys.
// Block (tile, limb r, work item w): work item = (product group, diagonals
// [i0, i1)); the tile holds 256*V consecutive evaluation indices (one half of
// the orbit order).  For each diagonal the key limbs (b_j, a_j)[r][t] are
// loaded once and applied to every product of the group that has it:
//   acc0_p += pt_{p,i} (P phi_i(c0_p) + sum_j phi_i(D_{p,j}) b_{i,j})
//   acc1_p += pt_{p,i} (                sum_j phi_i(D_{p,j}) a_{i,j})
// phi_i is a shift by i inside the orbit half, so every digit (and P c0) row
// a work item reads is the window [t0 + i0, t0 + tile + i1) of that row: it
// is staged in LDS once and the shifted reads of the loop become LDS reads.
// Partial sums per (product, chunk) go to part[prod.part0 + i0 / CH].
// ---------------------------------------------------------------------------
typedef double dbl2 __attribute__((ext_vector_type(2)));


template <int PG, int BETA, int V>
__global__ __launch_bounds__(256) void k_diag_batch(BatchDiagArgs a) {
  extern __shared__ double stage[];  // [PG][BETA + 1][win]
  constexpr int TILE = 256 * V;
  // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous range of the task list so that tasks sharing a key tile (same
  // chunk, tile and limb, different product groups) run on one L2.
  const int bid = blockIdx.x;
  const int vt = (bid & 7) * a.per_xcd + (bid >> 3);
  if (vt >= a.n_tasks) return;
  const DiagTask task = a.tasks[vt];
  const int r = task.limb;
  const DiagWork w = a.work[task.work];
  const DiagGroup& G = a.groups[w.grp];
  const int N = a.N, half = N >> 1, K = a.K;
  const int t0 = task.tile * TILE;
  const int tl = threadIdx.x * V;        // first local index of this thread
  const size_t limbN = (size_t)r * N;
  const int pi = a.limb_prime[r];
  const int klimb = a.key_limb[r];
  const bool isq = r <= a.lv;
  const ModQ m = a.mods[pi];
  const int np = G.np;
  // Staged row layout.  With V = 2 a thread reads elements 2 tid + s and
  // 2 tid + s + 1: stride 2 across the wave, two lanes on every LDS bank.
  // The rows hold even and odd elements in separate halves instead (element
  // x at (x & 1) hw + x / 2), so every read of the loop is stride 1.
  const int hw = (TILE + a.CH + 1) / 2;
  const int win = V == 2 ? 2 * hw : TILE + a.CH;  // row stride (doubles)
  auto spos = [&](int x) { return V == 2 ? (x & 1) * hw + (x >> 1) : x; };
  const int span = TILE + (w.i1 - w.i0);
  const size_t KN = (size_t)K * N;
  const size_t Qoff = (size_t)(a.lv + 1) * N;
  // stage the digit rows (and P c0 for the Q limbs) of every product
  for (int p = 0; p < np; ++p) {
    const int prod = G.prod[p];
    const double* dig = a.digits + (size_t)prod * a.dig_stride + limbN;
    const double* pc = a.pc + (size_t)prod * a.pc_stride + limbN;
    for (int j = 0; j <= BETA; ++j) {
      if (j == BETA && !isq) break;
      const double* src = (j < BETA) ? dig + (size_t)j * KN : pc;
      double* dst = stage + (size_t)(p * (BETA + 1) + j) * win;
      for (int x = threadIdx.x; x < span; x += 256)  // read once per task: streamed past L2 as well
        dst[spos(x)] = __builtin_nontemporal_load(gmem(src) + ((t0 & half) | ((t0 + w.i0 + x) & (half - 1))));
    }
  }
  __syncthreads();
  int mp[PG];
  const double* ptp[PG];
#pragma unroll
  for (int p = 0; p < PG; ++p) {
    if (p < np) {
      const BatchProd& B = a.prods[G.prod[p]];
      mp[p] = B.mprime;
      ptp[p] = B.pt + limbN + t0 + tl;
    } else {
      mp[p] = 0;
      ptp[p] = nullptr;
    }
  }
  double acc0[PG][V], acc1[PG][V];
#pragma unroll
  for (int p = 0; p < PG; ++p)
#pragma unroll
    for (int v = 0; v < V; ++v) acc0[p][v] = acc1[p][v] = 0.0;
  int cnt = 0;
  int i = w.i0;
  if (i == 0) {  // diagonal 0: no rotation; P c0 on the Q limbs
    if (isq) {
#pragma unroll
      for (int p = 0; p < PG; ++p) {
        if (p >= np) continue;
        const double* pcs = stage + (size_t)(p * (BETA + 1) + BETA) * win;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const double pv = gmem(ptp[p])[v];
          acc0[p][v] += mulmod(pv, pcs[spos(tl + v)], m);
          acc1[p][v] += mulmod(pv, gmem(a.pc)[(size_t)G.prod[p] * a.pc_stride + Qoff + limbN + t0 + tl + v], m);
        }
      }
    }
    ++i;
    ++cnt;
  }
  // key limbs (b_j, a_j) of rotation i at this thread's V indices
  // the key of rotation ii sits at slot slot_of_rot[ii] of the key set; the
  // loops read those slots one step ahead, so that no scalar-load wait stands
  // between a step's compute and the next step's loads
  auto slot_of = [&](int ii) { return a.slot_of_rot[min(ii, w.i1 - 1)]; };
  auto load_keys = [&](int slot, double (&kb)[BETA][V], double (&ka)[BETA][V]) {
    const auto* key = gmem(a.keys) + (size_t)slot * a.key_stride + (size_t)klimb * N + t0 + tl;
#pragma unroll
    for (int j = 0; j < BETA; ++j) {
      if (V == 2) {
        const dbl2 b2 = *(const __attribute__((address_space(1))) dbl2*)(key + (size_t)j * 2 * a.key_limbs * N);
        const dbl2 a2 = *(const __attribute__((address_space(1))) dbl2*)(key + (size_t)(j * 2 + 1) * a.key_limbs * N);
        kb[j][0] = b2.x; kb[j][V - 1] = b2.y;
        ka[j][0] = a2.x; ka[j][V - 1] = a2.y;
      } else {
        kb[j][0] = key[(size_t)j * 2 * a.key_limbs * N];
        ka[j][0] = key[(size_t)(j * 2 + 1) * a.key_limbs * N];
      }
    }
  };
  // plaintext values of diagonal i for every product of the group.  A
  // product without diagonal i (or an empty group slot) reads a row it has
  // and contributes zero, so the loads are unconditional and the two
  // diagonals' loads below can all be in flight together.  Plaintexts are
  // read once: stream them past L2 so that they do not evict the key tile
  // the other product groups of this chunk still need.
  auto load_pt = [&](int ii, double (&pv)[PG][V]) {
#pragma unroll
    for (int p = 0; p < PG; ++p) {
      const bool has = p < np && ii < mp[p];
      const double* src = ptp[p < np ? p : 0] + (size_t)(has ? ii : 0) * KN;
      if (V == 2) {
        const dbl2 p2 = __builtin_nontemporal_load(gmem((const dbl2*)src));
        pv[p][0] = has ? p2.x : 0.0;
        pv[p][V - 1] = has ? p2.y : 0.0;
      } else {
        const double x = __builtin_nontemporal_load(gmem(src));
        pv[p][0] = has ? x : 0.0;
      }
    }
  };
  auto apply = [&](int ii, const double (&kb)[BETA][V], const double (&ka)[BETA][V], const double (&pv)[PG][V]) {
    const int sh = ii - w.i0;  // shift of diagonal ii inside the window
#pragma unroll
    for (int p = 0; p < PG; ++p) {
      const double* st = stage + (size_t)(p * (BETA + 1)) * win;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        // spos(tl + sh + v), written out with tl = 2 tid for V = 2
        const int pos = V == 2 ? ((sh + v) & 1) * hw + (int)threadIdx.x + ((sh + v) >> 1) : tl + sh + v;
        // the sums start from their first term (adding it to 0.0 would cost an instruction)
        const double d0 = st[pos];
        double u0 = mulmod(d0, kb[0][v], m), u1 = mulmod(d0, ka[0][v], m);
#pragma unroll
        for (int j = 1; j < BETA; ++j) {
          const double d = st[(size_t)j * win + pos];
          u0 += mulmod(d, kb[j][v], m);
          u1 += mulmod(d, ka[j][v], m);
        }
        if (isq) u0 += st[(size_t)BETA * win + pos];
        acc0[p][v] += mulmod(pv[p][v], u0, m);
        acc1[p][v] += mulmod(pv[p][v], u1, m);
      }
    }
  };
  // re-centre after 8 (9 in the chunk holding diagonal 0) terms of |r| < q:
  // |acc| < 9.5 q < 2^52, the range reduce() takes
  auto settle = [&]() {
    if (cnt >= 8) {
#pragma unroll
      for (int p = 0; p < PG; ++p)
#pragma unroll
        for (int v = 0; v < V; ++v) {
          acc0[p][v] = reduce(acc0[p][v], m);
          acc1[p][v] = reduce(acc1[p][v], m);
        }
      cnt = 0;
    }
  };
  // (a chunk with no rotated diagonal may come with no key set at all)
  int sl0 = i < w.i1 ? slot_of(i) : 0, sl1 = i + 1 < w.i1 ? slot_of(i + 1) : 0;
  // two diagonals per step: both diagonals' key and plaintext loads are
  // issued before either is used, which doubles the memory requests each
  // wave has in flight (the LDS stage already limits occupancy to three
  // waves per SIMD, which leaves the registers for this)
  for (; i + 1 < w.i1; i += 2) {
    double kb0[BETA][V], ka0[BETA][V], kb1[BETA][V], ka1[BETA][V], pv0[PG][V], pv1[PG][V];
    load_keys(sl0, kb0, ka0);
    load_pt(i, pv0);
    load_keys(sl1, kb1, ka1);
    load_pt(i + 1, pv1);
    sl0 = slot_of(i + 2);
    sl1 = slot_of(i + 3);
    apply(i, kb0, ka0, pv0);
    apply(i + 1, kb1, ka1, pv1);
    cnt += 2;
    settle();
  }
  if (i < w.i1) {
    double kb0[BETA][V], ka0[BETA][V], pv0[PG][V];
    load_keys(sl0, kb0, ka0);
    load_pt(i, pv0);
    apply(i, kb0, ka0, pv0);
  }
  const int chunk = w.i0 / a.CH;
#pragma unroll
  for (int p = 0; p < PG; ++p) {
    if (p >= np || w.i0 >= mp[p]) continue;
    double* part = a.part + (size_t)(a.prods[G.prod[p]].part0 + chunk) * 2 * KN + limbN + t0 + tl;
#pragma unroll
    for (int v = 0; v < V; ++v) {  // summed by a later launch: keep them out of L2
      __builtin_nontemporal_store(reduce(acc0[p][v], m), part + v);
      __builtin_nontemporal_store(reduce(acc1[p][v], m), part + KN + v);
    }
  }
}

// acc[p] = sum of the chunk partials of product p;  acc [count][2][K][N]
__global__ __launch_bounds__(256) void k_sum_partials_batch(const double* __restrict__ part, const BatchProd* __restrict__ prods,
                                                           int CH, int K, int N, LimbMap limb_prime,
                                                           const ModQ* __restrict__ mods, double* __restrict__ acc) {
  const size_t tot = (size_t)2 * K * N;
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= tot) return;
  const int p = blockIdx.y;
  const BatchProd B = prods[p];
  const int nch = (B.mprime + CH - 1) / CH;
  const int r = (int)((idx / N) % K);
  const ModQ m = mods[limb_prime.idx[r]];
  // eight partials' loads in flight at a time, added in chunk order with a
  // re-centring after every eighth (|v| < 8.5 q): the per-call form's sum
  const double* src = part + (size_t)B.part0 * tot + idx;
  double v = 0.0;
  int c = 0;
  for (; c + 8 <= nch; c += 8) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = __builtin_nontemporal_load(gmem(src) + (size_t)(c + u) * tot);
#pragma unroll
    for (int u = 0; u < 8; ++u) v += t[u];
    v = reduce(v, m);
  }
  for (; c < nch; ++c) v += __builtin_nontemporal_load(gmem(src) + (size_t)c * tot);
  acc[(size_t)p * tot + idx] = reduce(v, m);
}

// Workgroups go round-robin over the 8 XCDs; each XCD takes a contiguous
// range of the (product, diagonal) list so that neighbouring diagonals of one
// product, which read neighbouring columns of X, share its L2.
template <int LOGN>
__global__ __launch_bounds__(NttShape<LOGN>::T) void k_encode_pt_batch(const EncodeArgs* __restrict__ args,
                                                                       const int2* __restrict__ work, int nwork,
                                                                       const BatchProd* __restrict__ prods, EncTabs et,
                                                                       LimbMap map, DevTabs tb) {
  __shared__ double2 s2[NttShape<LOGN>::LDS / 2];
  const int per_xcd = (nwork + 7) / 8;
  const int vt = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (vt >= nwork) return;
  const int2 wk = work[vt];
  const EncodeArgs a = args[wk.x];
  double* out = prods[wk.x].pt_out + (size_t)wk.y * map.n * (1 << LOGN);
  encode_pt_body<LOGN>(a, wk.y, et, map, tb, s2, out);
}

template <int LOGN>
__global__ __launch_bounds__(NttShape<LOGN>::T) void k_encode_ct_batch(const EncodeArgs* __restrict__ args, EncTabs et,
                                                                       int64_t* __restrict__ msg) {
  constexpr int N = 1 << LOGN, T = NttShape<LOGN>::T, PH = N / 2 / T;
  __shared__ double2 s2[NttShape<LOGN>::LDS / 2];
  const int c = blockIdx.x;
  double mreg[2 * PH];
  const EncodeArgs a = args[c];
  encode_to_regs<LOGN, true>(a, 0, s2, mreg, et, a.scale);
  int64_t* dst = msg + (size_t)c * N;
#pragma unroll
  for (int u = 0; u < PH; ++u) {
    const int kk = threadIdx.x + u * T;
    dst[kk] = (int64_t)mreg[2 * u];
    dst[kk + N / 2] = (int64_t)mreg[2 * u + 1];
  }
}

// read-out of product p's decoded slots z[p][N/2] into its y (lazy RaS)
// output row idx of a product from its decoded slots slot(j): the lazy
// rotate-and-sum, added in slot order
template <class Slot>
__device__ __forceinline__ double readout_row(const EncodeArgs& a, int idx, Slot slot) {
  double acc = 0.0;
  if (a.kind == 0) {
    const int rr = idx, g = rr / a.mprime, rho = rr % a.mprime;
    for (int t2 = 0; t2 < a.bn / a.mprime; ++t2) acc += slot(g * a.bn + rho + t2 * a.mprime);
  } else if (a.bm >= a.bn) {
    acc = slot(idx);
  } else {
    for (int t2 = 0; t2 < a.bn / a.bm; ++t2) acc += slot(idx + t2 * a.bm);
  }
  return acc;
}

__global__ __launch_bounds__(256) void k_readout_batch(const double* __restrict__ z, const EncodeArgs* __restrict__ args,
                                                       const BatchProd* __restrict__ prods, int slots) {
  const int p = blockIdx.y;
  const EncodeArgs a = args[p];
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= a.m) return;
  const double* zp = z + (size_t)p * slots;
  prods[p].y[idx] = readout_row(a, idx, [&](int j) { return zp[j]; });
}

// Decode and read-out in one workgroup per product (N <= 2^14): the slots
// stay in LDS and each row's sum reads them there.  Same values and the same
// order of additions as k_decode followed by k_readout_batch.
template <int LOGN>
__global__ __launch_bounds__(NttShape<LOGN>::T) void k_decode_readout_batch(const double* __restrict__ res, int lv,
                                                                            CrtTabs ct, EncTabs et, double inv_scale,
                                                                            const EncodeArgs* __restrict__ args,
                                                                            const BatchProd* __restrict__ prods) {
  constexpr int N = 1 << LOGN, T = NttShape<LOGN>::T;
  __shared__ double2 w[NttShape<LOGN>::LDS / 2];
  const int p = blockIdx.x;
  decode_to_lds<LOGN>(res + (size_t)p * (lv + 1) * N, lv + 1, ct, et, w);
  const EncodeArgs a = args[p];
  double* y = prods[p].y;
  for (int idx = threadIdx.x; idx < a.m; idx += T)
    y[idx] = readout_row(a, idx, [&](int j) { return decoded_slot<LOGN>(w, et, j, inv_scale); });
}

// ---------------------------------------------------------------------------
#define DISPATCH_LOGN(L, FN, ...)                         \
  switch ((L).logN) {                                     \
    case 12: FN<12>(__VA_ARGS__); break;                  \
    case 13: FN<13>(__VA_ARGS__); break;                  \
    case 14: FN<14>(__VA_ARGS__); break;                  \
    case 15: FN<15>(__VA_ARGS__); break;                  \
    default: return hipErrorInvalidValue;                 \
  }

template <int PG, int V>
static hipError_t diag_batch_pgv(const LaunchCtx& L, const BatchDiagArgs& a, int beta) {
  const dim3 grid(8 * a.per_xcd);
  const size_t lds = sizeof(double) * (size_t)PG * (beta + 1) * (256 * V + a.CH + 1);  // row stride <= win + 1
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  switch (beta) {
    case 1: hipLaunchKernelGGL((k_diag_batch<PG, 1, V>), grid, dim3(256), lds, L.stream, a); break;
    case 2: hipLaunchKernelGGL((k_diag_batch<PG, 2, V>), grid, dim3(256), lds, L.stream, a); break;
    case 3: hipLaunchKernelGGL((k_diag_batch<PG, 3, V>), grid, dim3(256), lds, L.stream, a); break;
    case 4: hipLaunchKernelGGL((k_diag_batch<PG, 4, V>), grid, dim3(256), lds, L.stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// dynamic LDS above the default limit must be opted in per kernel instance
template <int PG, int V>
static hipError_t diag_batch_allow_lds() {
  const int bytes = 160 * 1024;
  const void* fn[4] = {(const void*)k_diag_batch<PG, 1, V>, (const void*)k_diag_batch<PG, 2, V>,
                       (const void*)k_diag_batch<PG, 3, V>, (const void*)k_diag_batch<PG, 4, V>};
  for (const void* f : fn) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_diag_batch(const LaunchCtx& L, const BatchDiagArgs& a, int pg, int beta, int vec) {
  if (a.n_tasks <= 0) return hipSuccess;
  static bool lds_opt_in = false;
  if (!lds_opt_in) {
    const hipError_t e[6] = {diag_batch_allow_lds<1, 1>(), diag_batch_allow_lds<2, 1>(), diag_batch_allow_lds<4, 1>(),
                             diag_batch_allow_lds<1, 2>(), diag_batch_allow_lds<2, 2>(), diag_batch_allow_lds<4, 2>()};
    for (hipError_t x : e)
      if (x != hipSuccess) return x;
    lds_opt_in = true;
  }
  if (a.N % (256 * vec) != 0) return hipErrorInvalidValue;
  if (vec == 1) {
    switch (pg) {
      case 1: return diag_batch_pgv<1, 1>(L, a, beta);
      case 2: return diag_batch_pgv<2, 1>(L, a, beta);
      case 4: return diag_batch_pgv<4, 1>(L, a, beta);
    }
  } else if (vec == 2) {
    switch (pg) {
      case 1: return diag_batch_pgv<1, 2>(L, a, beta);
      case 2: return diag_batch_pgv<2, 2>(L, a, beta);
      case 4: return diag_batch_pgv<4, 2>(L, a, beta);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sum_partials_batch(const LaunchCtx& L, const double* part, const BatchProd* prods, int count, int CH,
                                     int K, int N, LimbMap limb_prime, double* acc) {
  const size_t tot = (size_t)2 * K * N;
  hipLaunchKernelGGL(k_sum_partials_batch, dim3((unsigned)((tot + 255) / 256), count), dim3(256), 0, L.stream, part, prods,
                     CH, K, N, limb_prime, L.tb.mods, acc);
  return hipGetLastError();
}

template <int LOGN>
static void enc_pt_batch_impl(const LaunchCtx& L, const EncodeArgs* args, const int2* work, int nwork,
                              const BatchProd* prods, const EncTabs& et, LimbMap map) {
  hipLaunchKernelGGL(k_encode_pt_batch<LOGN>, dim3(8 * ((nwork + 7) / 8)), dim3(NttShape<LOGN>::T), 0, L.stream, args,
                     work, nwork, prods, et, map, L.tb);
}
hipError_t launch_encode_pt_batch(const LaunchCtx& L, const EncodeArgs* args, const int2* work, int nwork,
                                  const BatchProd* prods, const EncTabs& et, LimbMap map) {
  if (nwork <= 0) return hipSuccess;
  DISPATCH_LOGN(L, enc_pt_batch_impl, L, args, work, nwork, prods, et, map);
  return hipGetLastError();
}

template <int LOGN>
static void enc_ct_batch_impl(const LaunchCtx& L, const EncodeArgs* args, int count, const EncTabs& et, int64_t* msg) {
  hipLaunchKernelGGL(k_encode_ct_batch<LOGN>, dim3(count), dim3(NttShape<LOGN>::T), 0, L.stream, args, et, msg);
}
hipError_t launch_encode_ct_batch(const LaunchCtx& L, const EncodeArgs* args, int count, const EncTabs& et, int64_t* msg) {
  DISPATCH_LOGN(L, enc_ct_batch_impl, L, args, count, et, msg);
  return hipGetLastError();
}

template <int LOGN>
static void decode_readout_impl(const LaunchCtx& L, const double* res, int count, int lv, const CrtTabs& ct,
                                const EncTabs& et, double inv_scale, const EncodeArgs* args, const BatchProd* prods) {
  if constexpr (LOGN <= 14)
    hipLaunchKernelGGL(k_decode_readout_batch<LOGN>, dim3(count), dim3(NttShape<LOGN>::T), 0, L.stream, res, lv, ct, et,
                       inv_scale, args, prods);
}
hipError_t launch_decode_readout_batch(const LaunchCtx& L, const double* res, int count, int lv, const CrtTabs& ct,
                                       const EncTabs& et, double inv_scale, const EncodeArgs* args,
                                       const BatchProd* prods) {
  if (L.logN > 14) return hipErrorInvalidValue;
  DISPATCH_LOGN(L, decode_readout_impl, L, res, count, lv, ct, et, inv_scale, args, prods);
  return hipGetLastError();
}
hipError_t launch_readout_batch(const LaunchCtx& L, const double* z, const EncodeArgs* args, const BatchProd* prods,
                                int count, int max_rows, int slots) {
  hipLaunchKernelGGL(k_readout_batch, dim3((max_rows + 255) / 256, count), dim3(256), 0, L.stream, z, args, prods, slots);
  return hipGetLastError();
}

}  // namespace pvfl
