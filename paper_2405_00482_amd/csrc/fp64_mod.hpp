// Exact modular arithmetic on binary64 for primes q < 2^48 (gfx950 VALU).
//
// Residues are integers held exactly in IEEE-754 binary64 (|x| < 2^53).  On
// CDNA4 the FP64 FMA and round-to-integer instructions issue at full rate,
// while a 64x64-bit integer product costs many 32-bit multiply steps, so the
// ring arithmetic of RNS-CKKS is carried out with this exact scheme:
//
//   h = a*b (rounded), l = fma(a, b, -h)          =>  a*b = h + l exactly
//   k = rint(h * (1/q))                           (quotient estimate)
//   r = fma(-k, q, h) + l                         =>  r = a*b - k*q exactly
//
// fma(-k, q, h) is exact because its result is an integer of magnitude below
// 2^53, and r + l is exact for the same reason.  The quotient estimate has
// relative error below 3 * 2^-53, so with |a*b/q| < 2^50 (e.g. |a| <= 2^51,
// |b| <= q/2 + 1) k is within 0.875 of a*b/q and |r| < q.  Every function
// states the input range it needs and the output range it gives.
// Compile with -ffp-contract=off: contraction would change h and break the
// identity a*b = h + l.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pvfl {

struct ModQ {
  double q;     // the prime, exact
  double qinv;  // 1/q rounded to nearest
};

// a*b mod q as some representative r with |r| < q.
// Needs |a*b/q| < 2^50 (e.g. |a| <= 4q, |b| <= q/2 + 1).
__device__ __forceinline__ double mulmod(double a, double b, ModQ m) {
  double h = a * b;
  double l = __builtin_fma(a, b, -h);
  double k = __builtin_rint(h * m.qinv);
  double r = __builtin_fma(-k, m.q, h);
  return r + l;
}

// centred representative, |r| <= (q+1)/2, for any integer |x| < 2^52.
__device__ __forceinline__ double reduce(double x, ModQ m) {
  double k = __builtin_rint(x * m.qinv);
  return __builtin_fma(-k, m.q, x);
}

// least non-negative residue in [0, q), for any integer |x| < 2^52.
__device__ __forceinline__ double canon(double x, ModQ m) {
  double r = reduce(x, m);
  r = (r < 0.0) ? r + m.q : r;
  return (r >= m.q) ? r - m.q : r;
}

// u64 in [0, 2^52) <-> binary64, two instructions each way.
__device__ __forceinline__ double u64_to_f64(uint64_t x) {
  return __longlong_as_double((long long)(x | 0x4330000000000000ull)) - 4503599627370496.0;
}
__device__ __forceinline__ uint64_t f64_to_u64(double c) {  // c integer in [0, 2^52)
  return (uint64_t)__double_as_longlong(c + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
}

// signed 64-bit integer -> centred residue (|m| may be up to 2^63).
__device__ __forceinline__ double i64_to_res(int64_t v, ModQ m, double two32_mod) {
  // v = hi * 2^32 + lo with lo in [0, 2^32): both parts exact in binary64
  int64_t hi = v >> 32;
  double lo = (double)(uint32_t)(v & 0xffffffffll);
  double h = reduce((double)hi, m);
  double t = mulmod(h, two32_mod, m);
  return reduce(t + lo, m);
}

}  // namespace pvfl
