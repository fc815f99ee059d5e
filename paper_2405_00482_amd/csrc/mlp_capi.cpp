// C ABI of the latency-model MLP (pvfl_mlp_*).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <random>
#include <vector>

#include "capi_internal.hpp"
#include "mlp.hpp"

using namespace pvfl;

#define HIP_TRY(expr)                                          \
  do {                                                         \
    hipError_t _e = (expr);                                    \
    if (_e != hipSuccess) return hip_fail(_e, #expr);          \
  } while (0)

struct pvfl_mlp {
  int F = 0, H = 0, n_params = 0, max_batch = 0;
  int64_t steps = 0;
  float *params = nullptr, *m = nullptr, *v = nullptr, *g = nullptr, *gs = nullptr, *lb = nullptr, *loss = nullptr;
  ~pvfl_mlp() {
    for (float* p : {params, m, v, g, gs, lb, loss})
      if (p) (void)hipFree(p);
  }
};

static int mlp_param_count(int F, int H) { return H * F + H + H * H + H + H + 1; }

extern "C" pvfl_status pvfl_mlp_create(int32_t n_in, int32_t hidden, int32_t max_batch, uint64_t seed, pvfl_mlp** out) {
  if (!out || n_in < 1 || n_in > kMlpMaxIn || hidden < 1 || hidden > kMlpMaxHidden || max_batch < 1)
    return fail(PVFL_E_INVALID, "mlp sizes out of range");
  std::unique_ptr<pvfl_mlp> n(new pvfl_mlp());
  n->F = n_in;
  n->H = hidden;
  n->max_batch = max_batch;
  n->n_params = mlp_param_count(n_in, hidden);
  const size_t P = n->n_params;
  for (float** p : {&n->params, &n->m, &n->v, &n->g})
    if (hipMalloc((void**)p, P * sizeof(float)) != hipSuccess) return fail(PVFL_E_NOMEM, "mlp allocation");
  if (hipMalloc((void**)&n->gs, P * max_batch * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&n->lb, max_batch * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&n->loss, sizeof(float)) != hipSuccess)
    return fail(PVFL_E_NOMEM, "mlp allocation");
  // He-uniform initialisation of the weights, zero biases
  std::mt19937_64 rng(seed);
  std::vector<float> h(P, 0.f);
  auto fill = [&](size_t off, int fan_in, int count) {
    const float lim = std::sqrt(6.f / (float)fan_in);
    std::uniform_real_distribution<float> d(-lim, lim);
    for (int i = 0; i < count; ++i) h[off + i] = d(rng);
  };
  const int F = n_in, H = hidden;
  fill(0, F, H * F);
  fill((size_t)H * F + H, H, H * H);
  fill((size_t)H * F + H + H * H + H, H, H);
  HIP_TRY(hipMemcpy(n->params, h.data(), P * sizeof(float), hipMemcpyHostToDevice));
  std::vector<float> z(P, 0.f);
  HIP_TRY(hipMemcpy(n->m, z.data(), P * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(n->v, z.data(), P * sizeof(float), hipMemcpyHostToDevice));
  *out = n.release();
  return PVFL_OK;
}

extern "C" void pvfl_mlp_destroy(pvfl_mlp* n) { delete n; }

extern "C" int32_t pvfl_mlp_num_params(const pvfl_mlp* n) { return n ? n->n_params : 0; }

extern "C" pvfl_status pvfl_mlp_get_params(const pvfl_mlp* n, float* out_dev, void* stream) {
  if (!n || !out_dev) return fail(PVFL_E_INVALID, "null argument");
  HIP_TRY(hipMemcpyAsync(out_dev, n->params, n->n_params * sizeof(float), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_mlp_set_params(pvfl_mlp* n, const float* in_dev, void* stream) {
  if (!n || !in_dev) return fail(PVFL_E_INVALID, "null argument");
  HIP_TRY(hipMemcpyAsync(n->params, in_dev, n->n_params * sizeof(float), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_mlp_forward(const pvfl_mlp* n, const float* x_dev, int32_t batch, float* y_dev,
                                        void* stream) {
  if (!n || !x_dev || !y_dev || batch < 0) return fail(PVFL_E_INVALID, "bad argument");
  HIP_TRY(launch_mlp_forward((hipStream_t)stream, n->params, n->F, n->H, x_dev, batch, y_dev));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_mlp_grad(pvfl_mlp* n, const float* x_dev, const float* t_dev, int32_t batch,
                                     float* grad_dev, float* loss_dev, void* stream) {
  if (!n || !x_dev || !t_dev || batch < 1) return fail(PVFL_E_INVALID, "bad argument");
  if (batch > n->max_batch) return fail(PVFL_E_SHAPE, "batch larger than the network's max_batch");
  HIP_TRY(launch_mlp_grad((hipStream_t)stream, n->params, n->F, n->H, x_dev, t_dev, batch, n->gs, n->lb, n->n_params,
                          grad_dev ? grad_dev : n->g, loss_dev ? loss_dev : n->loss));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_mlp_train_step(pvfl_mlp* n, const float* x_dev, const float* t_dev, int32_t batch,
                                           float lr, float* loss_dev, void* stream) {
  if (!n || !x_dev || !t_dev || batch < 1) return fail(PVFL_E_INVALID, "bad argument");
  if (batch > n->max_batch) return fail(PVFL_E_SHAPE, "batch larger than the network's max_batch");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_mlp_grad(s, n->params, n->F, n->H, x_dev, t_dev, batch, n->gs, n->lb, n->n_params, n->g,
                          loss_dev ? loss_dev : n->loss));
  n->steps += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - std::pow(b1, (float)n->steps), c2 = 1.f - std::pow(b2, (float)n->steps);
  HIP_TRY(launch_mlp_adam(s, n->params, n->m, n->v, n->g, n->n_params, lr, b1, b2, eps, c1, c2));
  return PVFL_OK;
}
