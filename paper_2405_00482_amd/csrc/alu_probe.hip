// Arithmetic-throughput probes behind the choice of exact binary64 modular
// arithmetic: how many modular products per second gfx950 sustains when the
// residues are held as doubles (q < 2^48, the exact-product-plus-rounded-
// quotient form of fp64_mod.hpp) and when they are held as 64-bit integers
// (q < 2^62, Shoup's precomputed-quotient form, whose 64x64-bit products the
// hardware builds from 32-bit multiplies), plus the raw FP64 FMA and 32-bit
// integer multiply rates.  Every thread runs 8 independent dependency chains
// so that issue rate, not latency, bounds each probe; the chains' final
// values are stored so nothing is optimised away.  Measurement only: nothing
// on the product path calls these kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fp64_mod.hpp"

namespace {

constexpr int kChains = 8;

__global__ __launch_bounds__(256) void k_fp64_fma(double* out, int iters, double a, double b) {
  double x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = (double)(threadIdx.x + c);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = __builtin_fma(x[c], a, b);
  }
  double s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_fp64_mulmod(double* out, int iters, double w, pvfl::ModQ m) {
  double x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = (double)(threadIdx.x * 7919 + c * 104729);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = pvfl::mulmod(x[c], w, m);
  }
  double s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Shoup: r = a w - floor(a w' / 2^64) q with w' = floor(w 2^64 / q), then one
// conditional subtraction (q < 2^62)
__global__ __launch_bounds__(256) void k_u64_shoup(uint64_t* out, int iters, uint64_t w, uint64_t wq, uint64_t q) {
  uint64_t x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = (uint64_t)threadIdx.x * 7919u + (uint64_t)c * 104729u;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      const uint64_t hi = __umul64hi(x[c], wq);
      uint64_t r = x[c] * w - hi * q;
      x[c] = r >= q ? r - q : r;
    }
  }
  uint64_t s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s ^= x[c];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 64 x 64 -> 128-bit product (low and high words), the core of any 64-bit
// integer modular product
__global__ __launch_bounds__(256) void k_u64_mul128(uint64_t* out, int iters, uint64_t w) {
  uint64_t x[kChains], h[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    x[c] = (uint64_t)threadIdx.x * 7919u + (uint64_t)c * 104729u + 1u;
    h[c] = 0;
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      h[c] ^= __umul64hi(x[c], w);
      x[c] = x[c] * w + 1u;
    }
  }
  uint64_t s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s ^= x[c] ^ h[c];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_u32_mul(uint32_t* out, int iters, uint32_t w) {
  uint32_t x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = threadIdx.x * 7919u + (uint32_t)c * 104729u + 1u;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = x[c] * w + 1u;
  }
  uint32_t s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s ^= x[c];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

// probe: 0 FP64 FMA, 1 FP64 modular product, 2 u64 Shoup modular product,
// 3 u64 128-bit product, 4 u32 multiply-add.  `out` holds blocks * 256
// 8-byte words.  Returns the number of operations of the launch (chains x
// iterations x threads), or -1 for an unknown probe or a launch error.
extern "C" double pvfl_probe_alu(int probe, int blocks, int iters, void* out, void* stream) {
  const dim3 grid(blocks), block(256);
  hipStream_t s = (hipStream_t)stream;
  const uint64_t q = (1ull << 61) - 1;           // a modulus below 2^62 (Shoup's form needs no primality)
  const uint64_t w = 0x1234567890abcull % q;
  const uint64_t wq = (uint64_t)(((unsigned __int128)w << 64) / q);
  const double qd = 281474976694273.0;           // a prime below 2^48
  const pvfl::ModQ m{qd, 1.0 / qd};
  switch (probe) {
    case 0: hipLaunchKernelGGL(k_fp64_fma, grid, block, 0, s, (double*)out, iters, 0.999999, 1e-7); break;
    case 1: hipLaunchKernelGGL(k_fp64_mulmod, grid, block, 0, s, (double*)out, iters, 123456789012.0, m); break;
    case 2: hipLaunchKernelGGL(k_u64_shoup, grid, block, 0, s, (uint64_t*)out, iters, w, wq, q); break;
    case 3: hipLaunchKernelGGL(k_u64_mul128, grid, block, 0, s, (uint64_t*)out, iters, w | 1u); break;
    case 4: hipLaunchKernelGGL(k_u32_mul, grid, block, 0, s, (uint32_t*)out, iters, 2654435761u); break;
    default: return -1.0;
  }
  if (hipGetLastError() != hipSuccess) return -1.0;
  return (double)kChains * iters * blocks * 256.0;
}
