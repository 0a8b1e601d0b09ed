// Refinement helpers: mean-squared query error against brute-force targets and
// one Adam step on the factor tables (not part of the paper's method).
#include <math.h>

#include "common.h"

namespace {

__global__ void k_zero_scalar(double* __restrict__ p) { p[0] = 0.0; }

__global__ __launch_bounds__(256) void k_mse_grad(int64_t nq, const float* __restrict__ q,
                                                  const double* __restrict__ target,
                                                  float* __restrict__ gout, double* __restrict__ loss) {
  __shared__ double sh[4];
  const double inv = 1.0 / static_cast<double>(nq);
  double acc = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < nq;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double d = static_cast<double>(q[i]) - target[i];
    gout[i] = static_cast<float>(2.0 * d * inv);
    acc += d * d;
  }
  if (!loss) return;
  acc = glint_wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, (sh[0] + sh[1] + sh[2] + sh[3]) * inv);
}

__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

}  // namespace

extern "C" {

glint_status glint_mse_grad(int64_t nq, const float* q, const double* target, float* gout,
                            double* loss, hipStream_t stream) {
  GLINT_REQUIRE(nq >= 1, "nq must be >= 1");
  GLINT_REQUIRE(q && target && gout, "null pointer argument");
  glint_clear_launch_error();
  if (loss) {
    hipLaunchKernelGGL(k_zero_scalar, dim3(1), dim3(1), 0, stream, loss);
    GLINT_LAUNCHED("k_zero_scalar");
  }
  const int64_t blocks = (nq + 255) / 256 < 2048 ? (nq + 255) / 256 : 2048;
  hipLaunchKernelGGL(k_mse_grad, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, nq, q,
                     target, gout, loss);
  GLINT_LAUNCHED("k_mse_grad");
  return GLINT_OK;
}

glint_status glint_adam_step(int64_t n, float* p, const float* g, float* m, float* v, float lr,
                             float b1, float b2, float eps, int32_t step, hipStream_t stream) {
  GLINT_REQUIRE(n >= 1 && step >= 1, "n and step must be >= 1");
  GLINT_REQUIRE(p && g && m && v, "null pointer argument");
  const float c1 = static_cast<float>(1.0 - pow(static_cast<double>(b1), step));
  const float c2 = static_cast<float>(1.0 - pow(static_cast<double>(b2), step));
  const int64_t blocks = (n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048;
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, n, p, g, m, v,
                     lr, b1, b2, eps, c1, c2);
  GLINT_LAUNCHED("k_adam");
  return GLINT_OK;
}

}  // extern "C"
