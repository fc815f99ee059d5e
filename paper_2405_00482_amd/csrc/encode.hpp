// Encoder/decoder argument structures (canonical embedding, plan packing).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace pvfl {

struct EncTabs {
  const uint32_t* slot2f;   // [N/2] slot j -> DFT index f_j = (5^j mod 2N - 1) / 4
  const uint32_t* f2slot;   // [N/2] the inverse permutation
  const double2* fft_tw;    // [N/4] exp(-2 pi i t / (N/2))
  const double2* twist;     // [N/2] zeta^k = exp(i pi k / N)
};

struct CrtTabs {
  const ModQ* mods;
  const double* garner_inv; // [kMaxLimbs][kMaxLimbs]: q_j^-1 mod q_i (centred), j < i
};

// Plan geometry as the packing kernels see it (all sizes padded to 2^k).
struct EncodeArgs {
  int kind;        // 0 HYBRID, 1 DIAG, 2 ROW, 3 CTMAT
  int m, n, ld;    // operand shape; ld = row stride of X (elements)
  const double* X; // plaintext matrix (pt encode) or encrypted operand (ct encode)
  int bm, bn, mprime, col_blocks, width, pack, n_out, n_out_cts, slots;
  int lbn, lmp, lw;  // log2 of bn, mprime, width (all powers of two)
  double scale;    // encoding scale
  double ind_scale;  // ROW: scale of the indicator plaintext
  int bsgs;          // HYBRID: baby-step size; diagonal i is stored rotated right by (i / bsgs) * bsgs
};

// per-limb factors (centred residues) of a plaintext encoded at a lower scale
struct OutFactors {
  double f[kMaxLimbs];
};

hipError_t launch_encode_pt(const LaunchCtx& L, const EncodeArgs& a, const EncTabs& et, LimbMap map, int count,
                            double* out);
// cleartext at the plan's output scale (pvfl_encode_out): out[count][map.n][N]
hipError_t launch_encode_out(const LaunchCtx& L, const EncodeArgs& a, const double* v, int mode, int ras_in_ct,
                             const OutFactors& fac, const EncTabs& et, LimbMap map, int count, double* out);
// out c0 = ct c0 + sign * pt (c1 copied) on nct ciphertexts
hipError_t launch_out_add_pt(const LaunchCtx& L, const double* ct, const double* pt, double sign, int nct, int lv, int N,
                             double* out);
hipError_t launch_encode_ct(const LaunchCtx& L, const EncodeArgs& a, const EncTabs& et, int count, int64_t* msg);
hipError_t launch_decode(const LaunchCtx& L, const double* res, int nct, int lv, const CrtTabs& ct, const EncTabs& et,
                         double inv_scale, double* z);
hipError_t launch_readout(const LaunchCtx& L, const double* z, const EncodeArgs& a, int ras_in_ct, int count, double* y);

}  // namespace pvfl
