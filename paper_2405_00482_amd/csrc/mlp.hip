// Latency-model network of the plan selector: a 3-layer perceptron
//   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3
// in FP32 with hand-written forward, backward and Adam kernels.  The sizes
// are tiny (F <= 64 inputs, H <= 64 hidden), so one workgroup of H threads
// handles one sample: thread u owns hidden unit u of both layers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp.hpp"

namespace pvfl {

// parameter layout: W1[H][F], b1[H], W2[H][H], b2[H], w3[H], b3
struct MlpView {
  float *W1, *b1, *W2, *b2, *w3, *b3;
};
__device__ __forceinline__ MlpView mlp_view(float* p, int F, int H) {
  MlpView v;
  v.W1 = p;
  v.b1 = v.W1 + H * F;
  v.W2 = v.b1 + H;
  v.b2 = v.W2 + H * H;
  v.w3 = v.b2 + H;
  v.b3 = v.w3 + H;
  return v;
}

// forward for one sample per workgroup; writes y[b]
__global__ __launch_bounds__(kMlpMaxHidden) void k_mlp_forward(const float* __restrict__ params, int F, int H,
                                                               const float* __restrict__ x, int B, float* __restrict__ y) {
  __shared__ float xs[kMlpMaxIn], h1[kMlpMaxHidden], h2[kMlpMaxHidden];
  const int b = blockIdx.x, u = threadIdx.x;
  if (b >= B) return;
  const MlpView P = mlp_view((float*)params, F, H);
  for (int f = u; f < F; f += blockDim.x) xs[f] = x[(size_t)b * F + f];
  __syncthreads();
  if (u < H) {
    float a = P.b1[u];
    for (int f = 0; f < F; ++f) a += P.W1[u * F + f] * xs[f];
    h1[u] = a > 0.f ? a : 0.f;
  }
  __syncthreads();
  if (u < H) {
    float a = P.b2[u];
    for (int k = 0; k < H; ++k) a += P.W2[u * H + k] * h1[k];
    h2[u] = a > 0.f ? a : 0.f;
  }
  __syncthreads();
  if (u == 0) {
    float a = P.b3[0];
    for (int k = 0; k < H; ++k) a += P.w3[k] * h2[k];
    y[b] = a;
  }
}

// per-sample gradient of L = (1/B) sum_b (y_b - t_b)^2, written to
// gs[b][n_params]; loss contribution to lb[b]
__global__ __launch_bounds__(kMlpMaxHidden) void k_mlp_backward(const float* __restrict__ params, int F, int H,
                                                                const float* __restrict__ x, const float* __restrict__ t,
                                                                int B, float* __restrict__ gs, float* __restrict__ lb,
                                                                int n_params) {
  __shared__ float xs[kMlpMaxIn], z1[kMlpMaxHidden], h1[kMlpMaxHidden], z2[kMlpMaxHidden], h2[kMlpMaxHidden];
  __shared__ float d2[kMlpMaxHidden], dy;
  const int b = blockIdx.x, u = threadIdx.x;
  if (b >= B) return;
  const MlpView P = mlp_view((float*)params, F, H);
  MlpView G = mlp_view(gs + (size_t)b * n_params, F, H);
  for (int f = u; f < F; f += blockDim.x) xs[f] = x[(size_t)b * F + f];
  __syncthreads();
  if (u < H) {
    float a = P.b1[u];
    for (int f = 0; f < F; ++f) a += P.W1[u * F + f] * xs[f];
    z1[u] = a;
    h1[u] = a > 0.f ? a : 0.f;
  }
  __syncthreads();
  if (u < H) {
    float a = P.b2[u];
    for (int k = 0; k < H; ++k) a += P.W2[u * H + k] * h1[k];
    z2[u] = a;
    h2[u] = a > 0.f ? a : 0.f;
  }
  __syncthreads();
  if (u == 0) {
    float a = P.b3[0];
    for (int k = 0; k < H; ++k) a += P.w3[k] * h2[k];
    const float r = a - t[b];
    lb[b] = r * r / (float)B;
    dy = 2.f * r / (float)B;
    G.b3[0] = dy;
  }
  __syncthreads();
  if (u < H) {
    G.w3[u] = dy * h2[u];
    d2[u] = (z2[u] > 0.f) ? dy * P.w3[u] : 0.f;
    G.b2[u] = d2[u];
    for (int k = 0; k < H; ++k) G.W2[u * H + k] = d2[u] * h1[k];
  }
  __syncthreads();
  if (u < H) {
    float a = 0.f;
    for (int v = 0; v < H; ++v) a += P.W2[v * H + u] * d2[v];
    const float d1 = (z1[u] > 0.f) ? a : 0.f;
    G.b1[u] = d1;
    for (int f = 0; f < F; ++f) G.W1[u * F + f] = d1 * xs[f];
  }
}

// g[p] = sum_b gs[b][p]; loss = sum_b lb[b] (written by thread 0 of block 0)
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ gs, const float* __restrict__ lb, int B,
                                                    int n_params, float* __restrict__ g, float* __restrict__ loss) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < n_params) {
    float a = 0.f;
    for (int b = 0; b < B; ++b) a += gs[(size_t)b * n_params + p];
    g[p] = a;
  }
  if (p == 0 && loss) {
    float a = 0.f;
    for (int b = 0; b < B; ++b) a += lb[b];
    *loss = a;
  }
}

// Adam (Kingma & Ba 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr * mhat / (sqrt(vhat) + eps)
__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ params, float* __restrict__ m, float* __restrict__ v,
                                                  const float* __restrict__ g, int n_params, float lr, float beta1,
                                                  float beta2, float eps, float corr1, float corr2) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n_params) return;
  const float gp = g[p];
  const float mp = beta1 * m[p] + (1.f - beta1) * gp;
  const float vp = beta2 * v[p] + (1.f - beta2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  params[p] -= lr * (mp / corr1) / (sqrtf(vp / corr2) + eps);
}

hipError_t launch_mlp_forward(hipStream_t s, const float* params, int F, int H, const float* x, int B, float* y) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3(B), dim3(kMlpMaxHidden), 0, s, params, F, H, x, B, y);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(hipStream_t s, const float* params, int F, int H, const float* x, const float* t, int B,
                           float* gs, float* lb, int n_params, float* g, float* loss) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_backward, dim3(B), dim3(kMlpMaxHidden), 0, s, params, F, H, x, t, B, gs, lb, n_params);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((n_params + 255) / 256), dim3(256), 0, s, gs, lb, B, n_params, g, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(hipStream_t s, float* params, float* m, float* v, const float* g, int n_params, float lr,
                           float beta1, float beta2, float eps, float corr1, float corr2) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((n_params + 255) / 256), dim3(256), 0, s, params, m, v, g, n_params, lr, beta1,
                     beta2, eps, corr1, corr2);
  return hipGetLastError();
}

}  // namespace pvfl
