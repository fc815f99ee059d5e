// Latency-model MLP of the plan selector (kernels in mlp.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace pvfl {
constexpr int kMlpMaxIn = 64;
constexpr int kMlpMaxHidden = 64;
hipError_t launch_mlp_forward(hipStream_t s, const float* params, int F, int H, const float* x, int B, float* y);
hipError_t launch_mlp_grad(hipStream_t s, const float* params, int F, int H, const float* x, const float* t, int B,
                           float* gs, float* lb, int n_params, float* g, float* loss);
hipError_t launch_mlp_adam(hipStream_t s, float* params, float* m, float* v, const float* g, int n_params, float lr,
                           float beta1, float beta2, float eps, float corr1, float corr2);
}  // namespace pvfl
