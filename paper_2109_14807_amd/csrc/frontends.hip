// Query front-ends built on the range query.
//
// Environment-light prefiltering (Sec. 5.4): a spherical-Gaussian light lobe
// G(w) = A exp(lambda (cos w - 1)) exceeds eps exactly within its compact-eps
// support angle theta = arccos((ln eps - ln A) / lambda + 1); the NDF is
// averaged over the square of side N theta / pi bins (the projected
// half-vector square spans pi radians) centred on the lookup's half vector.
#include <cmath>
#include <cstdint>

#include "common.h"

namespace {

constexpr int kSgThreads = 256;

// Half-open bin range of the continuous extent [h - w/2, h + w/2] of the
// projected square [-1, 1] (FP64; clamped before the conversion to int).
__device__ __forceinline__ void sg_bins(double h, double w, int N, int& lo, int& hi) {
  const double half_n = 0.5 * N;
  const double a = floor((h - 0.5 * w + 1.0) * half_n);
  const double b = floor((h + 0.5 * w + 1.0) * half_n);
  lo = static_cast<int>(fmin(fmax(a, 0.0), static_cast<double>(N - 1)));
  hi = static_cast<int>(fmin(fmax(b, 0.0), static_cast<double>(N - 1))) + 1;
}

__global__ __launch_bounds__(kSgThreads) void k_sg_records(int64_t n, int N, double log_eps,
                                                           const int32_t* __restrict__ uvl,
                                                           const float* __restrict__ h,
                                                           const float* __restrict__ sg,
                                                           int32_t* __restrict__ q) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double lam = static_cast<double>(sg[2 * i]), amp = static_cast<double>(sg[2 * i + 1]);
  double arg = (log_eps - log(amp)) / lam + 1.0;
  if (!isfinite(arg)) arg = 1.0;                      // not a valid lobe: point lookup
  const double theta = acos(fmin(fmax(arg, -1.0), 1.0));
  const double w = fmin(2.0 * theta / M_PI, 2.0);
  double hs = static_cast<double>(h[2 * i]), ht = static_cast<double>(h[2 * i + 1]);
  if (!isfinite(hs)) hs = 0.0;
  if (!isfinite(ht)) ht = 0.0;
  int slo, shi, tlo, thi;
  sg_bins(hs, w, N, slo, shi);
  sg_bins(ht, w, N, tlo, thi);
  int32_t* r = q + 7 * i;
  r[0] = uvl[3 * i];
  r[1] = uvl[3 * i + 1];
  r[2] = uvl[3 * i + 2];
  r[3] = slo;
  r[4] = shi;
  r[5] = tlo;
  r[6] = thi;
}

__global__ __launch_bounds__(kSgThreads) void k_box_average(int64_t n, const int32_t* __restrict__ q,
                                                            float* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t* r = q + 7 * i;
  const int area = (r[4] - r[3]) * (r[6] - r[5]);     // >= 1 by construction
  out[i] = out[i] / static_cast<float>(area);
}

}  // namespace

extern "C" {

glint_status glint_query_sg(const glint_factors* f, int64_t n, const int32_t* uvl, const float* h,
                            const float* sg, float eps, int32_t* q, float* out, hipStream_t stream) {
  GLINT_REQUIRE(f != nullptr, "factors are NULL");
  GLINT_REQUIRE(n >= 0, "n must be >= 0");
  GLINT_REQUIRE(std::isfinite(eps) && eps > 0.0f, "eps must be finite and positive");
  GLINT_REQUIRE(f->nbins >= 1, "factors have no bins");
  if (n == 0) return GLINT_OK;
  GLINT_REQUIRE(uvl && h && sg && q && out, "null pointer argument");
  const unsigned blocks = static_cast<unsigned>((n + kSgThreads - 1) / kSgThreads);
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_sg_records, dim3(blocks), dim3(kSgThreads), 0, stream, n, f->nbins,
                     std::log(static_cast<double>(eps)), uvl, h, sg, q);
  GLINT_LAUNCHED("k_sg_records");
  const glint_status st = glint_query(f, n, q, out, stream);
  if (st != GLINT_OK) return st;
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_box_average, dim3(blocks), dim3(kSgThreads), 0, stream, n, q, out);
  GLINT_LAUNCHED("k_box_average");
  return GLINT_OK;
}

}  // extern "C"
