// Query front-ends built on the range query.
//
// Wang tiles (Sec. 5.5): the plane is a grid of S x S cells whose tiles come
// from hashed vertex edge colours and an edge-to-tile map, with no index map;
// each tile's CP covers footprint centres reaching m texels past the tile,
// with only the tile's texels contributing, so a footprint's range query is
// the sum of its overlapped cells' tile queries at its local centre.
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

// ---- Wang tiles ------------------------------------------------------------

constexpr int kWangThreads = 256;

struct WangArgs {
  int ntiles, S, m, P, R, nl, N;
  uint64_t seed;
  uint8_t etl[16];
  const float* U;
  const float* V;
  const float* L;
  const float* CS;
  const float* CT;
  int64_t nq;
  const int32_t* q;
  float* out;
};

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {
  return a >= 0 ? a / b : -((-a + b - 1) / b);
}

// colour of the edge to the right of vertex (i, j) (e = 0) or below it (e = 1)
__device__ __forceinline__ int edge_colour(uint64_t seed, int64_t i, int64_t j, int e) {
  const uint64_t c = ((((static_cast<uint64_t>(i) & 0xFFFFFFFFull) << 32) | (static_cast<uint64_t>(j) & 0xFFFFFFFFull))
                      << 1) | static_cast<uint64_t>(e);
  return glint_sm64_uniform(seed, c) >= 0.5 ? 1 : 0;
}

// one query per thread: the footprint's cells, each cell's tile, its CP query
__global__ __launch_bounds__(kWangThreads) void k_query_wang(WangArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.nq) return;
  const int32_t* r = a.q + 7 * i;
  const int64_t x = r[0], y = r[1];
  const int l = glint_clampi(r[2], 0, a.nl - 1);
  const int slo = glint_clampi(r[3], 0, a.N), shi = glint_clampi(r[4], 0, a.N);
  const int tlo = glint_clampi(r[5], 0, a.N), thi = glint_clampi(r[6], 0, a.N);
  float acc = 0.0f;
  if (slo < shi && tlo < thi) {
    const int64_t k = int64_t{1} << l;
    const int64_t x0 = x - k / 2, y0 = y - k / 2;
    const int64_t ci0 = floor_div(x0, a.S), ci1 = floor_div(x0 + k - 1, a.S);
    const int64_t cj0 = floor_div(y0, a.S), cj1 = floor_div(y0 + k - 1, a.S);
    for (int64_t ci = ci0; ci <= ci1; ++ci) {
      for (int64_t cj = cj0; cj <= cj1; ++cj) {
        const int top = edge_colour(a.seed, ci, cj, 0), left = edge_colour(a.seed, ci, cj, 1);
        const int right = edge_colour(a.seed, ci + 1, cj, 1), bottom = edge_colour(a.seed, ci, cj + 1, 0);
        const int tile = a.etl[8 * top + 4 * right + 2 * bottom + left];
        const int lu = static_cast<int>(x - ci * a.S + a.m), lv = static_cast<int>(y - cj * a.S + a.m);
        const float* U = a.U + (static_cast<int64_t>(tile) * a.P + lu) * a.R;
        const float* V = a.V + (static_cast<int64_t>(tile) * a.P + lv) * a.R;
        const float* L = a.L + (static_cast<int64_t>(tile) * a.nl + l) * a.R;
        const float* CS = a.CS + static_cast<int64_t>(tile) * (a.N + 1) * a.R;
        const float* CT = a.CT + static_cast<int64_t>(tile) * (a.N + 1) * a.R;
        // four ranks per 16-byte load (R % 4 == 0, tables 16-byte aligned),
        // added in rank order
        const float4* U4 = reinterpret_cast<const float4*>(U);
        const float4* V4 = reinterpret_cast<const float4*>(V);
        const float4* L4 = reinterpret_cast<const float4*>(L);
        const float4* SH = reinterpret_cast<const float4*>(CS + shi * a.R);
        const float4* SL = reinterpret_cast<const float4*>(CS + slo * a.R);
        const float4* TH = reinterpret_cast<const float4*>(CT + thi * a.R);
        const float4* TL = reinterpret_cast<const float4*>(CT + tlo * a.R);
        for (int r4 = 0; r4 < a.R / 4; ++r4) {
          const float4 u = U4[r4], v = V4[r4], w = L4[r4], sh = SH[r4], sl = SL[r4], th = TH[r4], tl = TL[r4];
          acc += u.x * v.x * w.x * (sh.x - sl.x) * (th.x - tl.x);
          acc += u.y * v.y * w.y * (sh.y - sl.y) * (th.y - tl.y);
          acc += u.z * v.z * w.z * (sh.z - sl.z) * (th.z - tl.z);
          acc += u.w * v.w * w.w * (sh.w - sl.w) * (th.w - tl.w);
        }
      }
    }
  }
  a.out[i] = acc;
}

// ---- record validation ---------------------------------------------------

constexpr int kValThreads = 256;

__global__ void k_zero_count(unsigned long long* n) {
  if (threadIdx.x == 0) *n = 0ull;
}

// A record is invalid when the query's rules would change it: u or v outside
// the map, l outside [0, nl), a bin bound outside [0, N], or lo > hi.
__global__ __launch_bounds__(kValThreads) void k_validate(int64_t nq, const int32_t* __restrict__ q, int nu, int nv,
                                                          int nl, int N, unsigned long long* __restrict__ nbad) {
  unsigned long long count = 0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i0 = static_cast<int64_t>(blockIdx.x) * blockDim.x; i0 < nq; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    bool bad = false;
    if (i < nq) {
      const int32_t* r = q + 7 * i;
      bad = r[0] < 0 || r[0] >= nu || r[1] < 0 || r[1] >= nv || r[2] < 0 || r[2] >= nl;
#pragma unroll
      for (int k = 3; k < 7; ++k) bad = bad || r[k] < 0 || r[k] > N;
      bad = bad || r[3] > r[4] || r[5] > r[6];
    }
    count += static_cast<unsigned long long>(__popcll(__ballot(bad)));
  }
  if ((threadIdx.x & 63) == 0 && count) atomicAdd(nbad, count);
}

}  // namespace

extern "C" {

glint_status glint_validate_queries(const glint_factors* f, int64_t nq, const int32_t* q, int64_t* nbad,
                                    hipStream_t stream) {
  GLINT_REQUIRE(f != nullptr && nbad != nullptr, "null pointer argument");
  GLINT_REQUIRE(f->nu >= 1 && f->nv >= 1 && f->nl >= 1 && f->nbins >= 1, "bad table sizes");
  GLINT_REQUIRE(nq >= 0, "nq must be >= 0");
  GLINT_REQUIRE(nq == 0 || q != nullptr, "null query pointer");
  unsigned long long* n = reinterpret_cast<unsigned long long*>(nbad);
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(64), 0, stream, n);
  GLINT_LAUNCHED("k_zero_count");
  if (nq == 0) return GLINT_OK;
  int64_t blocks = (nq + kValThreads - 1) / kValThreads;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_validate, dim3(static_cast<unsigned>(blocks)), dim3(kValThreads), 0, stream, nq, q, f->nu,
                     f->nv, f->nl, f->nbins, n);
  GLINT_LAUNCHED("k_validate");
  return GLINT_OK;
}


glint_status glint_query_wang(const glint_wang* w, int64_t nq, const int32_t* q, float* out, hipStream_t stream) {
  GLINT_REQUIRE(w != nullptr, "tile set is NULL");
  GLINT_REQUIRE(w->ntiles >= 1 && w->ntiles <= 256, "ntiles must be in [1, 256]");
  GLINT_REQUIRE(w->S >= 1 && w->m >= 0 && w->R >= 1 && w->nl >= 1 && w->nl <= 24 && w->nbins >= 1,
                "bad tile-set sizes");
  GLINT_REQUIRE(w->R % 4 == 0, "R %d must be a multiple of 4", w->R);
  GLINT_REQUIRE((int64_t{1} << (w->nl - 1)) <= 2 * static_cast<int64_t>(w->m),
                "the margin m must be at least half the largest footprint (2m >= 2^(nl-1))");
  GLINT_REQUIRE((int64_t{1} << (w->nl - 1)) <= static_cast<int64_t>(w->S),
                "tiles must be at least as wide as the largest footprint (2^(nl-1) <= S)");
  for (int c = 0; c < 16; ++c)
    GLINT_REQUIRE(w->edge_to_tile[c] < w->ntiles, "edge_to_tile[%d] = %d is not a tile", c, w->edge_to_tile[c]);
  GLINT_REQUIRE(nq >= 0, "nq must be >= 0");
  if (nq == 0) return GLINT_OK;
  GLINT_REQUIRE(w->U && w->V && w->L && w->CS && w->CT && q && out, "null pointer argument");
  GLINT_REQUIRE(glint_aligned(w->U, 16) && glint_aligned(w->V, 16) && glint_aligned(w->L, 16) &&
                    glint_aligned(w->CS, 16) && glint_aligned(w->CT, 16),
                "tile tables must be 16-byte aligned");
  WangArgs a;
  a.ntiles = w->ntiles; a.S = w->S; a.m = w->m; a.P = w->S + 2 * w->m; a.R = w->R; a.nl = w->nl; a.N = w->nbins;
  a.seed = w->seed;
  for (int c = 0; c < 16; ++c) a.etl[c] = w->edge_to_tile[c];
  a.U = w->U; a.V = w->V; a.L = w->L; a.CS = w->CS; a.CT = w->CT; a.nq = nq; a.q = q; a.out = out;
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_query_wang, dim3(static_cast<unsigned>((nq + kWangThreads - 1) / kWangThreads)),
                     dim3(kWangThreads), 0, stream, a);
  GLINT_LAUNCHED("k_query_wang");
  return GLINT_OK;
}


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
