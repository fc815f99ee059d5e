// Plan selection for both operand forms of the product.
//
// X (m x n) times an encrypted vector: every valid combination of plan kind
// (HYBRID, DIAG, ROW; Sec. 3-4), ModDown placement (lazy / per rotation) and
// rotation schedule (all rotations hoisted, or a baby-step/giant-step split
// with baby step b).  [[A]] (m x n) times W (n x n_out): Alg. 3 with every
// column-packing factor, or W^T times each encrypted row of A (a batch of m
// HYBRID or DIAG products sharing one plaintext set).  Two latency models
// rank them:
//
//  * analytic: the Table 2 operation counts of the plan (Mult, Add, Rot,
//    HstRot) plus the ModUp / ModDown counts and the number of encoded
//    plaintext limbs, each weighted by a per-operation latency the caller
//    measured for this parameter set;
//  * learned: the latency network (mlp.hip) maps the plan's feature vector to
//    log-latency; it is trained on measured plan latencies.
//
// The feature vector is fixed here so that the training data and the runtime
// choice agree.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "capi_internal.hpp"

using namespace pvfl;

#define HIP_TRY(expr)                                          \
  do {                                                         \
    hipError_t _e = (expr);                                    \
    if (_e != hipSuccess) return hip_fail(_e, #expr);          \
  } while (0)

namespace {
constexpr int kFeatures = PVFL_PLAN_FEATURES;
constexpr int kMaxCandidates = 64;
constexpr int kMaxBatchDigits = 4;  // digits the batched fused kernel is instantiated for

float lg1p(double x) { return (float)std::log2(1.0 + x); }

int ilog2i(int x) {
  int r = 0;
  while ((1 << r) < x) ++r;
  return r;
}

void features_of(const pvfl_plan* p, int batch, float* f) {
  const pvfl_plan_info& I = p->info;
  const pvfl_ctx* c = p->ctx;
  int k = 0;
  f[k++] = (float)c->logN;
  f[k++] = (float)(p->lv + 1);
  f[k++] = (float)c->alpha;
  f[k++] = (float)p->beta;
  f[k++] = (float)p->K;
  f[k++] = (float)ilog2i(I.m_pad);
  f[k++] = (float)ilog2i(I.n_pad);
  f[k++] = (float)ilog2i(std::max(1, I.mprime));
  f[k++] = I.kind == PVFL_PLAN_HYBRID ? 1.f : 0.f;
  f[k++] = I.kind == PVFL_PLAN_DIAG ? 1.f : 0.f;
  f[k++] = I.kind == PVFL_PLAN_ROW ? 1.f : 0.f;
  f[k++] = I.kind == PVFL_PLAN_CTMAT ? 1.f : 0.f;
  f[k++] = p->opts.lazy_moddown ? 1.f : 0.f;
  f[k++] = p->ras_rots.empty() ? 0.f : 1.f;
  f[k++] = I.bsgs ? 1.f : 0.f;
  f[k++] = I.bsgs ? (float)ilog2i(I.bsgs) : 0.f;
  f[k++] = I.kind == PVFL_PLAN_CTMAT ? (float)ilog2i(std::max(1, p->opts.pack)) : 0.f;
  f[k++] = (float)ilog2i(std::max(1, batch));
  f[k++] = lg1p((double)I.n_mult);
  f[k++] = lg1p((double)I.n_add);
  f[k++] = lg1p((double)I.n_rot);
  f[k++] = lg1p((double)I.n_hstrot);
  f[k++] = lg1p((double)I.n_modup);
  f[k++] = lg1p((double)I.n_moddown);
  f[k++] = lg1p((double)I.n_pts * I.pt_limbs);
  f[k++] = lg1p((double)I.n_galois);
  f[k++] = lg1p((double)I.row_blocks * I.col_blocks);
  // k == kFeatures
}

// every option set for X (m x n) times an encrypted vector at `level`
void enumerate_vec(pvfl_ctx* c, int m, int n, int level, std::vector<pvfl_plan_opts>& out) {
  auto base = [&](int kind) {
    pvfl_plan_opts o{};
    o.kind = kind;
    o.m = m;
    o.n = n;
    o.level = level;
    o.pack = 1;
    return o;
  };
  // HYBRID: lazy and per-rotation ModDown, hoisted; lazy with every baby step
  for (int lazy = 1; lazy >= 0; --lazy) {
    pvfl_plan_opts o = base(PVFL_PLAN_HYBRID);
    o.lazy_moddown = lazy;
    out.push_back(o);
  }
  {
    const int S = c->N / 2;
    const int mp = std::min(S, 1 << ilog2i(m)), np = std::min(S, 1 << ilog2i(n));
    const int mprime = std::max(1, (int)((int64_t)mp * np / S));
    for (int b = 2; 2 * b <= mprime; b *= 2) {
      pvfl_plan_opts o = base(PVFL_PLAN_HYBRID);
      o.lazy_moddown = 1;
      o.bsgs = b;
      out.push_back(o);
    }
  }
  // DIAG: lazy / per-rotation ModDown with lazy RaS; lazy with in-ciphertext RaS when m < n
  for (int lazy = 1; lazy >= 0; --lazy) {
    pvfl_plan_opts o = base(PVFL_PLAN_DIAG);
    o.lazy_moddown = lazy;
    out.push_back(o);
  }
  if (m < n) {
    pvfl_plan_opts o = base(PVFL_PLAN_DIAG);
    o.lazy_moddown = 1;
    o.ras_in_ct = 1;
    out.push_back(o);
  }
  out.push_back(base(PVFL_PLAN_ROW));
}

// [[A]] (m x n) times W (n x n_out): Alg. 3 with packing 1, 2, 4, ... as far as
// it fits, and the per-row form (W^T, n_out x n, times each row of A)
void enumerate_mat(pvfl_ctx* c, int m, int n, int n_out, int level, std::vector<pvfl_candidate>& out) {
  const int S = c->N / 2;
  const int width = std::max(1 << ilog2i(m), 1 << ilog2i(n));
  for (int pack = 1; (int64_t)pack * width <= S; pack *= 2) {
    pvfl_candidate k{};
    k.opts.kind = PVFL_PLAN_CTMAT;
    k.opts.m = m;
    k.opts.n = n;
    k.opts.n_out = n_out;
    k.opts.level = level;
    k.opts.pack = pack;
    k.batch = 1;
    out.push_back(k);
  }
  for (int kind : {PVFL_PLAN_HYBRID, PVFL_PLAN_DIAG}) {
    pvfl_candidate k{};
    k.opts.kind = kind;
    k.opts.m = n_out;
    k.opts.n = n;
    k.opts.level = level;
    k.opts.lazy_moddown = 1;
    k.opts.pack = 1;
    k.batch = m;
    out.push_back(k);
  }
}
}  // namespace

struct pvfl_planner {
  pvfl_mlp* mlp = nullptr;  // borrowed
  float x_mean[kFeatures], x_std[kFeatures];
  float y_mean = 0, y_std = 1;
  float* x_dev = nullptr;   // [kMaxCandidates][kFeatures]
  float* y_dev = nullptr;   // [kMaxCandidates]
  ~pvfl_planner() {
    if (x_dev) (void)hipFree(x_dev);
    if (y_dev) (void)hipFree(y_dev);
  }
};

extern "C" int32_t pvfl_plan_num_features(void) { return kFeatures; }

extern "C" pvfl_status pvfl_plan_features(const pvfl_plan* p, int32_t batch, float* out, int32_t cap) {
  if (!p || !out) return fail(PVFL_E_INVALID, "null argument");
  if (cap < kFeatures) return fail(PVFL_E_SHAPE, "feature buffer too small");
  if (batch < 1) return fail(PVFL_E_INVALID, "batch must be positive");
  features_of(p, batch, out);
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_plan_candidates(pvfl_ctx* c, int32_t operand, int32_t m, int32_t n, int32_t n_out,
                                            int32_t level, pvfl_candidate* out, int32_t cap, int32_t* count) {
  if (!c || !count || (!out && cap > 0)) return fail(PVFL_E_INVALID, "null argument");
  if (m < 1 || n < 1) return fail(PVFL_E_SHAPE, "m and n must be positive");
  std::vector<pvfl_candidate> all, ok;
  if (operand == PVFL_OPERAND_CT_VEC) {
    std::vector<pvfl_plan_opts> v;
    enumerate_vec(c, m, n, level, v);
    for (const pvfl_plan_opts& o : v) all.push_back(pvfl_candidate{o, 1});
  } else if (operand == PVFL_OPERAND_CT_MAT) {
    if (n_out < 1) return fail(PVFL_E_SHAPE, "n_out must be positive");
    enumerate_mat(c, m, n, n_out, level, all);
  } else {
    return fail(PVFL_E_INVALID, "unknown operand form");
  }
  for (const pvfl_candidate& k : all) {
    pvfl_plan* p = nullptr;
    if (pvfl_plan_create(c, &k.opts, &p) == PVFL_OK) {
      // the per-row form runs as one batch, whose fused kernel takes up to 4 digits
      if (k.batch == 1 || p->beta <= kMaxBatchDigits) ok.push_back(k);
      pvfl_plan_destroy(p);
    }
  }
  *count = (int32_t)ok.size();
  if ((int32_t)ok.size() > cap) return fail(PVFL_E_SHAPE, "candidate buffer too small");
  std::copy(ok.begin(), ok.end(), out);
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_plan_analytic_ms(const pvfl_plan* p, int32_t batch, const double* costs, double* ms) {
  if (!p || !costs || !ms) return fail(PVFL_E_INVALID, "null argument");
  if (batch < 1) return fail(PVFL_E_INVALID, "batch must be positive");
  const pvfl_plan_info& I = p->info;
  const double B = (double)batch;
  const double counts[PVFL_COST_TERMS] = {B * I.n_mult,   B * I.n_add,     B * I.n_rot,
                                          B * I.n_hstrot, B * I.n_modup,   B * I.n_moddown,
                                          (double)I.n_pts * I.pt_limbs, 1.0};
  double t = 0;
  for (int i = 0; i < PVFL_COST_TERMS; ++i) t += counts[i] * costs[i];
  *ms = t;
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_planner_create(pvfl_mlp* mlp, const float* x_mean, const float* x_std, float y_mean,
                                           float y_std, pvfl_planner** out) {
  if (!out || !x_mean || !x_std) return fail(PVFL_E_INVALID, "null argument");
  if (mlp && pvfl_mlp_num_params(mlp) <= 0) return fail(PVFL_E_INVALID, "bad network");
  std::unique_ptr<pvfl_planner> pl(new pvfl_planner());
  pl->mlp = mlp;
  for (int i = 0; i < kFeatures; ++i) {
    if (!(x_std[i] > 0.f)) return fail(PVFL_E_INVALID, "feature scales must be positive");
    pl->x_mean[i] = x_mean[i];
    pl->x_std[i] = x_std[i];
  }
  if (!(y_std > 0.f)) return fail(PVFL_E_INVALID, "target scale must be positive");
  pl->y_mean = y_mean;
  pl->y_std = y_std;
  if (hipMalloc((void**)&pl->x_dev, sizeof(float) * kMaxCandidates * kFeatures) != hipSuccess ||
      hipMalloc((void**)&pl->y_dev, sizeof(float) * kMaxCandidates) != hipSuccess)
    return fail(PVFL_E_NOMEM, "planner buffers");
  *out = pl.release();
  return PVFL_OK;
}

extern "C" void pvfl_planner_destroy(pvfl_planner* pl) { delete pl; }

extern "C" pvfl_status pvfl_plan_choose(pvfl_planner* pl, pvfl_ctx* c, int32_t operand, int32_t m, int32_t n,
                                        int32_t n_out, int32_t level, const double* costs, pvfl_candidate* chosen,
                                        double* predicted_ms, void* stream) {
  if (!c || !chosen) return fail(PVFL_E_INVALID, "null argument");
  if (!costs && (!pl || !pl->mlp)) return fail(PVFL_E_INVALID, "neither a network nor operation costs given");
  std::vector<pvfl_candidate> cand(kMaxCandidates);
  int32_t nc = 0;
  pvfl_status st = pvfl_plan_candidates(c, operand, m, n, n_out, level, cand.data(), kMaxCandidates, &nc);
  if (st != PVFL_OK) return st;
  if (nc == 0) return fail(PVFL_E_PLAN, "no valid plan for this shape");
  std::vector<float> x((size_t)nc * kFeatures);
  std::vector<double> pred(nc);
  for (int i = 0; i < nc; ++i) {
    pvfl_plan* p = nullptr;
    if ((st = pvfl_plan_create(c, &cand[i].opts, &p)) != PVFL_OK) return st;
    features_of(p, cand[i].batch, &x[(size_t)i * kFeatures]);
    if (costs) pvfl_plan_analytic_ms(p, cand[i].batch, costs, &pred[i]);
    pvfl_plan_destroy(p);
  }
  if (!costs) {
    for (int i = 0; i < nc; ++i)
      for (int k = 0; k < kFeatures; ++k) {
        float& v = x[(size_t)i * kFeatures + k];
        v = (v - pl->x_mean[k]) / pl->x_std[k];
      }
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(pl->x_dev, x.data(), x.size() * sizeof(float), hipMemcpyHostToDevice, s));
    if ((st = pvfl_mlp_forward(pl->mlp, pl->x_dev, nc, pl->y_dev, stream)) != PVFL_OK) return st;
    std::vector<float> y(nc);
    HIP_TRY(hipMemcpyAsync(y.data(), pl->y_dev, nc * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < nc; ++i) pred[i] = std::exp((double)y[i] * pl->y_std + pl->y_mean);
  }
  const int best = (int)(std::min_element(pred.begin(), pred.end()) - pred.begin());
  *chosen = cand[best];
  if (predicted_ms) *predicted_ms = pred[best];
  return PVFL_OK;
}
