// Structures of the batched execution (many products, one launch per phase).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "encode.hpp"
#include "kernels.hpp"

namespace pvfl {

constexpr int kMaxGroup = 16;

struct BatchProd {
  const double* ct;   // input ciphertext [2][lv+1][N]
  const double* pt;   // diagonal plaintexts [mprime][K][N]
  double* pt_out;     // same buffer, writable (encoding)
  double* ct_out;     // input ciphertext, writable (encryption)
  double* out;        // output ciphertext [2][lv+1][N]
  double* y;          // decoded result
  int mprime;
  int part0;          // first partial-sum slot of this product
};

struct DiagGroup {
  int np;
  int prod[kMaxGroup];
};

struct DiagWork {
  int grp, i0, i1, pad;
};

// one workgroup of the fused kernel: work item, tile, limb
struct DiagTask {
  int work, tile, limb, pad;
};

struct BatchDiagArgs {
  int N, K, lv, key_limbs, CH;
  size_t key_stride;
  const ModQ* mods;
  int limb_prime[kMaxLimbs];
  int key_limb[kMaxLimbs];
  const BatchProd* prods;
  const DiagGroup* groups;
  const DiagWork* work;
  const DiagTask* tasks;   // [n_tasks], in the order they should share caches
  int n_tasks;
  int per_xcd;             // tasks per XCD (ceil(n_tasks / 8))
  const double* keys;
  const int* slot_of_rot;
  const double* digits;  // product p at digits + p * dig_stride, [beta][K][N]
  size_t dig_stride;
  const double* pc;      // product p at pc + p * pc_stride, [2][lv+1][N]
  size_t pc_stride;
  double* part;          // [slot][2][K][N]
};

// pg: products per group (1, 2, 4); vec: evaluation indices per thread (1, 2)
hipError_t launch_diag_batch(const LaunchCtx& L, const BatchDiagArgs& a, int pg, int beta, int vec);
hipError_t launch_sum_partials_batch(const LaunchCtx& L, const double* part, const BatchProd* prods, int count, int CH,
                                     int K, int N, LimbMap limb_prime, double* acc);
hipError_t launch_encode_pt_batch(const LaunchCtx& L, const EncodeArgs* args, const int2* work, int nwork,
                                  const BatchProd* prods, const EncTabs& et, LimbMap map);
hipError_t launch_encode_ct_batch(const LaunchCtx& L, const EncodeArgs* args, int count, const EncTabs& et, int64_t* msg);
// decode and lazy read-out of every product's decrypted residues (N <= 2^14)
hipError_t launch_decode_readout_batch(const LaunchCtx& L, const double* res, int count, int lv, const CrtTabs& ct,
                                       const EncTabs& et, double inv_scale, const EncodeArgs* args,
                                       const BatchProd* prods);
hipError_t launch_readout_batch(const LaunchCtx& L, const double* z, const EncodeArgs* args, const BatchProd* prods,
                                int count, int max_rows, int slots);

}  // namespace pvfl
