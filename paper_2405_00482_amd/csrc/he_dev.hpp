// Device helpers shared by the HIP kernel files: the counter-based
// generator and samplers, the orbit shift of a rotation, LDS write-out.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "ntt_core.hpp"

namespace pvfl {

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon et al., SC'11) and samplers.
// Word idx of stream `stream` under key `seed`: counter = (idx>>1, stream),
// key = seed, word (0,1) for even idx and (2,3) for odd idx, low word first.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t philox_word(uint64_t seed, uint64_t stream, uint64_t idx) {
  uint32_t c0 = (uint32_t)(idx >> 1), c1 = (uint32_t)(idx >> 33);
  uint32_t c2 = (uint32_t)stream, c3 = (uint32_t)(stream >> 32);
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return (idx & 1) ? ((uint64_t)c2 | ((uint64_t)c3 << 32)) : ((uint64_t)c0 | ((uint64_t)c1 << 32));
}

// floor(u * q / 2^64) for q < 2^49: the high 64 bits of a 64x64 product.
__device__ __forceinline__ uint64_t mul_hi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

__device__ __forceinline__ double sample_uniform_res(uint64_t seed, uint64_t stream, uint64_t idx, uint64_t q) {
  return u64_to_f64(mul_hi64(philox_word(seed, stream, idx), q));
}
__device__ __forceinline__ int sample_ternary(uint64_t seed, uint64_t stream, uint64_t idx) {
  return (int)mul_hi64(philox_word(seed, stream, idx), 3ull) - 1;
}
__device__ __forceinline__ int sample_cbd21(uint64_t seed, uint64_t stream, uint64_t idx) {
  const uint64_t u = philox_word(seed, stream, idx);
  return __popcll(u & 0x1FFFFFull) - __popcll((u >> 21) & 0x1FFFFFull);
}

__device__ __forceinline__ int orbit_shift(int t, int rot, int half) {
  return (t & half) | ((t + rot) & (half - 1));
}

}  // namespace pvfl
