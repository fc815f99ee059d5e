// Internal host-side objects behind the opaque handles of include/pvfl.h.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <string>
#include <vector>

#include "../../include/pvfl.h"
#include "kernels.hpp"

namespace pvfl {
typedef uint64_t u64;
u64 mulm(u64 a, u64 b, u64 q);
u64 powm(u64 a, u64 e, u64 q);
u64 invm(u64 a, u64 q);
double centred(u64 x, u64 q);
pvfl_status fail(pvfl_status s, const std::string& msg);
pvfl_status hip_fail(hipError_t e, const char* where);
}  // namespace pvfl

struct pvfl_ctx {
  int logN = 0, N = 0, n_q = 0, alpha = 0, device = 0;
  double log2_scale = 0;
  std::vector<pvfl::u64> primes;            // q_0..q_L, p_0..p_{alpha-1}
  std::vector<pvfl::ModQ> mods_host;
  pvfl::DevTabs tabs{};
  std::vector<int> log5;                    // discrete log base 5 mod 2N, -1 outside <5>
  std::vector<pvfl::KsLevel> ks_host;       // per level
  const pvfl::KsLevel* ks_dev = nullptr;    // [n_q]
  const double* pmod_dev = nullptr;         // P mod q_i, centred
  std::vector<pvfl::RescaleArgs> rescale;   // per level (index >= 1)
  std::vector<void*> dev_allocs;
  double* scratch = nullptr;
  size_t scratch_bytes = 0;
  // encoder tables (slot <-> FFT index, twiddles), created on first use
  void* enc_tabs = nullptr;
  void (*enc_tabs_free)(void*) = nullptr;
  // optional per-launch timing (HIP events on the launch stream)
  struct Timed {
    hipEvent_t start, stop;
    int cls;
    double bytes;
  };
  bool timing_on = false;
  std::vector<Timed> timed;
  ~pvfl_ctx();
};

struct pvfl_sk {
  pvfl_ctx* ctx = nullptr;
  double* s = nullptr;  // [n_mod][N]
  ~pvfl_sk();
};

struct pvfl_pk {
  pvfl_ctx* ctx = nullptr;
  double* pk = nullptr;  // [2][L+1][N]: b, then a (evaluation domain)
  ~pvfl_pk();
};

struct pvfl_rotkeys {
  pvfl_ctx* ctx = nullptr;
  int key_limbs = 0, beta = 0;
  size_t key_stride = 0;                // doubles per key
  double* keys = nullptr;               // [nkeys][beta][2][key_limbs][N]
  std::vector<uint32_t> galois;
  std::vector<int> rot;
  std::vector<int> slot_of_rot;         // [N/2] -> key index or -1
  int* slot_of_rot_dev = nullptr;
  ~pvfl_rotkeys();
};

namespace pvfl {
struct Term {
  int in_ct, rot, pt, out_ct;
};
}  // namespace pvfl

struct pvfl_plan {
  pvfl_ctx* ctx = nullptr;
  pvfl_plan_opts opts{};
  pvfl_plan_info info{};
  int lv = 0, K = 0, beta = 0;
  int bm = 0, bn = 0;          // block rows / columns (padded)
  double pt_scale = 0;         // Delta_pt
  std::vector<pvfl::Term> terms;
  std::vector<uint32_t> galois;
  // device tables
  int* iota_dev = nullptr;     // [max(mprime, 1)] = 0..mprime-1
  int* rot_dev = nullptr;      // BSGS: [mprime] baby rotation of diagonal i (i mod bsgs)
  int chunk = 1, nchunk = 1;   // diagonal chunking of the fused kernel (BSGS: nchunk = giant steps x chunks per step)
  int chunks_per_giant = 1;    // BSGS: chunks of one giant step's inner sum
  // DIAG plan: in-ciphertext RaS rotations; ROW plan: per-row data
  std::vector<int> ras_rots;
  ~pvfl_plan();
};

namespace pvfl {
// Set by entry points that must not create runtime objects (the
// allocation-free product): kernel timing is skipped for their launches.
inline thread_local bool t_timing_off = false;

// Brackets one kernel launch with HIP events when timing is enabled.
struct KernelTimer {
  pvfl_ctx* c;
  hipStream_t s;
  int cls;
  double bytes;
  hipEvent_t a = nullptr;
  KernelTimer(pvfl_ctx* c_, void* stream, int cls_, double bytes_) : c(c_), s((hipStream_t)stream), cls(cls_), bytes(bytes_) {
    if (c->timing_on && !t_timing_off && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, s);
  }
  void stop() {
    if (!a) return;
    hipEvent_t b;
    if (hipEventCreate(&b) == hipSuccess) {
      (void)hipEventRecord(b, s);
      c->timed.push_back(pvfl_ctx::Timed{a, b, cls, bytes});
    } else {
      (void)hipEventDestroy(a);
    }
    a = nullptr;
  }
};
LimbMap qp_map(const pvfl_ctx* c, int lv, bool with_p);
LimbMap key_limb_map(const pvfl_ctx* c, int lv);
LaunchCtx launch_ctx(const pvfl_ctx* c, void* stream);
pvfl_status ctx_scratch(pvfl_ctx* c, size_t bytes, double** out);
pvfl_status noalloc_scratch_init(int device);  // plan.cpp
pvfl_status keyswitch_digits(pvfl_ctx* c, const pvfl_rotkeys* keys, int lv, const double* digits, int rot_digits,
                             int key_rot, double* u, double* ydown, double* v, void* stream);
}  // namespace pvfl
