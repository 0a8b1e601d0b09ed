// NDF tensor of a normal map over every texel position and footprint level
// (Sec. 3.1 Eq. geom; Sec. 4.1), and the brute-force range integral.
//
//   k_texel_bins      one thread per (texel, axis): centre bin and the masses
//                     of the 2K+1 bins around it (FP64 erfc).
//   k_build_direct    level l from its footprint texels: a workgroup stages
//                     the bin windows of a k x (CB+k-1) texel tile in LDS and
//                     scatters each texel's (2K+1)^2 patch into an LDS block
//                     per cell; the block is written once, coalesced.
//   k_level_double    level l+1 = mean of four shifted level-l blocks (a 2k
//                     box is the union of two k boxes per axis), exact.
//   k_range_bruteforce one wave per query sums the footprint texels' window
//                     masses over the box.
#include <math.h>

#include <mutex>

#include "common.h"

namespace {

constexpr int kBuildThreads = 256;
constexpr size_t kStageBudget = 32768;   // LDS bytes for the texel tile
constexpr size_t kBlockBudget = 32768;   // LDS bytes for one cell's block strip

__global__ __launch_bounds__(256) void k_texel_bins(const float* __restrict__ nxy, int64_t n2,
                                                    int N, double sigma, int K,
                                                    int32_t* __restrict__ bins,
                                                    double* __restrict__ mass) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n2) return;
  const double n = static_cast<double>(nxy[idx]);
  const int P = 2 * K + 1;
  double* out = mass + idx * P;
  if (!isfinite(n)) {                // absent texel: no mass on this axis (so none at all)
    bins[idx] = 0;
    for (int j = 0; j < P; ++j) out[j] = 0.0;
    return;
  }
  const double halfN = 0.5 * static_cast<double>(N);
  int i0 = static_cast<int>(floor((n + 1.0) * halfN));
  i0 = glint_clampi(i0, 0, N - 1);
  bins[idx] = i0;
  const double w = 2.0 / static_cast<double>(N);
  const double zn = glint_gauss_interval((-1.0 - n) / sigma, (1.0 - n) / sigma);
  for (int j = 0; j < P; ++j) {
    const int i = i0 - K + j;
    double m = 0.0;
    if (i >= 0 && i < N) {
      const double e0 = -1.0 + static_cast<double>(i) * w;
      const double e1 = -1.0 + static_cast<double>(i + 1) * w;
      m = glint_gauss_interval((e0 - n) / sigma, (e1 - n) / sigma) / zn;
    }
    out[j] = m;
  }
}

// Direct build of one level for a strip of CB cells (u, v0 .. v0+CB-1).
// The output block of a cell is NO x NO bins, bins [s_off, s_off + NO) x
// [t_off, t_off + NO) of the NDF image (the whole image: offsets 0, NO = N).
// Dynamic LDS: [texels][2] bins | [texels][2][P] masses (OT) | block strip (OT).
template <typename OT>
__global__ __launch_bounds__(kBuildThreads) void k_build_direct(
    const int32_t* __restrict__ bins, const double* __restrict__ mass, int nu, int nv,
    int nlevels, int K, int level, int CB, int SR, int s_off, int t_off, int NO,
    OT* __restrict__ T) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int k = 1 << level;
  const int h = k >> 1;
  const int P = 2 * K + 1;
  const int W = CB + k - 1;
  const int ntex = k * W;
  int32_t* sbin = reinterpret_cast<int32_t*>(smem);
  OT* smass = reinterpret_cast<OT*>(smem + glint_round_up(sizeof(int32_t) * 2 * ntex, 16));
  OT* blk = reinterpret_cast<OT*>(reinterpret_cast<unsigned char*>(smass) +
                                  glint_round_up(sizeof(OT) * 2 * P * ntex, 16));

  const int u = blockIdx.y;
  const int v0 = blockIdx.x * CB;
  const int tid = threadIdx.x;

  // stage the tile's bin windows
  for (int idx = tid; idx < ntex; idx += blockDim.x) {
    const int i = idx / W, j = idx - (idx / W) * W;
    int x = (u - h + i) % nu;
    if (x < 0) x += nu;
    int y = (v0 - h + j) % nv;
    if (y < 0) y += nv;
    const int64_t tex = static_cast<int64_t>(x) * nv + y;
    sbin[2 * idx] = bins[2 * tex];
    sbin[2 * idx + 1] = bins[2 * tex + 1];
    const double* m = mass + tex * 2 * P;
    for (int a = 0; a < 2 * P; ++a) smass[idx * 2 * P + a] = static_cast<OT>(m[a]);
  }
  __syncthreads();

  const OT inv_area = static_cast<OT>(1.0 / (static_cast<double>(k) * k));
  const int ncell = min(CB, nv - v0);
  const int items = k * k * P * P;
  // the block strip in 16-byte words: zeroed once here, then every word is
  // zeroed again by the thread that writes it out
  constexpr int VEC = 16 / sizeof(OT);
  using V = typename std::conditional<sizeof(OT) == 4, float4, double2>::type;
  V* blk4 = reinterpret_cast<V*>(blk);
  const int strip4 = min(SR, NO) * NO / VEC;
  for (int e = tid; e < strip4; e += blockDim.x) blk4[e] = V{};
  __syncthreads();
  for (int c = 0; c < ncell; ++c) {
    const int v = v0 + c;
    OT* dst = T + ((static_cast<int64_t>(u) * nv + v) * nlevels + level) * NO * NO;
    for (int s0 = 0; s0 < NO; s0 += SR) {
      const int rows = min(SR, NO - s0);
      for (int it = tid; it < items; it += blockDim.x) {
        const int texi = it / (P * P);
        const int rem = it - texi * P * P;
        const int a = rem / P, b = rem - (rem / P) * P;
        const int fi = texi / k, fj = texi - (texi / k) * k;   // footprint row, column
        const int sidx = fi * W + (c + fj);
        const int s = sbin[2 * sidx] - K + a - s_off;
        const int t = sbin[2 * sidx + 1] - K + b - t_off;
        if (s >= s0 && s < s0 + rows && t >= 0 && t < NO) {
          const OT val = smass[sidx * 2 * P + a] * smass[sidx * 2 * P + P + b];
          if (val != OT(0)) atomicAdd(&blk[(s - s0) * NO + t], val);
        }
      }
      __syncthreads();
      V* d = reinterpret_cast<V*>(dst + static_cast<int64_t>(s0) * NO);
      const int n4 = rows * NO / VEC;
      for (int e = tid; e < n4; e += blockDim.x) {
        V x = blk4[e];
        blk4[e] = V{};
        x.x *= inv_area;
        x.y *= inv_area;
        if constexpr (VEC == 4) {
          x.z *= inv_area;
          x.w *= inv_area;
        }
        d[e] = x;
      }
      __syncthreads();
    }
  }
}

// Level l+1 from level l: T1(u,v) = 1/4 sum_{a in {u-ceil(k/2), u+floor(k/2)}}
//                                          sum_{b in {v-ceil(k/2), v+floor(k/2)}} T0(a,b).
template <typename OT>
__global__ __launch_bounds__(256) void k_level_double(OT* __restrict__ T, int nu, int nv,
                                                      int nlevels, int N, int level) {
  const int k = 1 << level;
  const int u = blockIdx.y, v = blockIdx.x;
  const int up = (k + 1) >> 1, dn = k >> 1;
  const int ua = (u - up + nu) % nu, ub = (u + dn) % nu;
  const int va = (v - up + nv) % nv, vb = (v + dn) % nv;
  const int64_t NN = static_cast<int64_t>(N) * N;
  auto blk = [&](int x, int y, int l) {
    return T + ((static_cast<int64_t>(x) * nv + y) * nlevels + l) * NN;
  };
  const OT* A = blk(ua, va, level);
  const OT* B = blk(ua, vb, level);
  const OT* C = blk(ub, va, level);
  const OT* D = blk(ub, vb, level);
  OT* O = blk(u, v, level + 1);
  constexpr int VEC = 16 / sizeof(OT);
  using V = typename std::conditional<sizeof(OT) == 4, float4, double2>::type;
  const int64_t nvec = NN / VEC;
  for (int64_t e = threadIdx.x; e < nvec; e += blockDim.x) {
    V a = reinterpret_cast<const V*>(A)[e];
    V b = reinterpret_cast<const V*>(B)[e];
    V c = reinterpret_cast<const V*>(C)[e];
    V d = reinterpret_cast<const V*>(D)[e];
    V o;
    const OT q = OT(0.25);
    o.x = ((a.x + b.x) + (c.x + d.x)) * q;
    o.y = ((a.y + b.y) + (c.y + d.y)) * q;
    if constexpr (VEC == 4) {
      o.z = ((a.z + b.z) + (c.z + d.z)) * q;
      o.w = ((a.w + b.w) + (c.w + d.w)) * q;
    }
    reinterpret_cast<V*>(O)[e] = o;
  }
}

// Level l+1 from level l for an m x m tile of output cells spaced k apart,
// (u0 + i k, v0 + j k): their sources are the (m+1) x (m+1) level-l blocks
// (u0 - ceil(k/2) + i k, v0 - ceil(k/2) + j k), each read once for up to four
// outputs (m = 4: 1.56 block reads per output instead of 4; m = 8: 1.27).  One thread per
// 16 bytes of a block, for every cell of its tile; the same sums as
// k_level_double.  Needs nu and nv to be multiples of m k.
template <typename OT, int M>
__global__ __launch_bounds__(256) void k_level_double_tile(OT* __restrict__ T, int nu, int nv, int nlevels,
                                                           int NN, int level) {
  constexpr int VEC = 16 / sizeof(OT);
  using V = typename std::conditional<sizeof(OT) == 4, float4, double2>::type;
  const int nvec = NN / VEC;
  const int k = 1 << level;
  const int up = (k + 1) >> 1;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t tile = idx / nvec;
  const int nsu = nu / (M * k), nsv = nv / (M * k);
  if (tile >= static_cast<int64_t>(nsu) * nsv * k * k) return;
  const int e = static_cast<int>(idx - tile * nvec);
  const int64_t ph = tile / (static_cast<int64_t>(nsu) * nsv);
  const int st = static_cast<int>(tile - ph * nsu * nsv);
  const int pu = static_cast<int>(ph / k), pv = static_cast<int>(ph % k);
  const int u0 = (st / nsv) * M * k + pu, v0 = (st % nsv) * M * k + pv;
  int xs[M + 1], ys[M + 1];
#pragma unroll
  for (int i = 0; i <= M; ++i) {
    xs[i] = ((u0 - up + i * k) % nu + nu) % nu;
    ys[i] = ((v0 - up + i * k) % nv + nv) % nv;
  }
  auto src = [&](int x, int y) {
    return reinterpret_cast<const V*>(T + ((static_cast<int64_t>(x) * nv + y) * nlevels + level) * NN)[e];
  };
  const OT q = OT(0.25);
  V prev[M + 1];
#pragma unroll
  for (int j = 0; j <= M; ++j) prev[j] = src(xs[0], ys[j]);
#pragma unroll
  for (int i = 1; i <= M; ++i) {
    V cur[M + 1];
#pragma unroll
    for (int j = 0; j <= M; ++j) cur[j] = src(xs[i], ys[j]);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      // A = (row i-1, col j), B = (row i-1, col j+1), C = (row i, col j), D = (row i, col j+1)
      const V a = prev[j], b = prev[j + 1], c = cur[j], d = cur[j + 1];
      V o;
      o.x = ((a.x + b.x) + (c.x + d.x)) * q;
      o.y = ((a.y + b.y) + (c.y + d.y)) * q;
      if constexpr (VEC == 4) {
        o.z = ((a.z + b.z) + (c.z + d.z)) * q;
        o.w = ((a.w + b.w) + (c.w + d.w)) * q;
      }
      const int u = u0 + (i - 1) * k, v = v0 + j * k;
      reinterpret_cast<V*>(T + ((static_cast<int64_t>(u) * nv + v) * nlevels + level + 1) * NN)[e] = o;
    }
#pragma unroll
    for (int j = 0; j <= M; ++j) prev[j] = cur[j];
  }
}

// The same for blocks of NN <= 1024 elements (the angular blocks of the
// clustered layout): one thread per 16 bytes of output over all cells, so a
// workgroup covers several cells instead of leaving most of its lanes idle.
template <typename OT>
__global__ __launch_bounds__(256) void k_level_double_flat(OT* __restrict__ T, int nu, int nv,
                                                           int nlevels, int NN, int level) {
  constexpr int VEC = 16 / sizeof(OT);
  using V = typename std::conditional<sizeof(OT) == 4, float4, double2>::type;
  const int nvec = NN / VEC;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t cell = idx / nvec;
  if (cell >= static_cast<int64_t>(nu) * nv) return;
  const int e = static_cast<int>(idx - cell * nvec);
  const int u = static_cast<int>(cell / nv), v = static_cast<int>(cell - static_cast<int64_t>(u) * nv);
  const int k = 1 << level;
  const int up = (k + 1) >> 1, dn = k >> 1;
  const int ua = (u - up + nu) % nu, ub = (u + dn) % nu;
  const int va = (v - up + nv) % nv, vb = (v + dn) % nv;
  auto blk = [&](int x, int y, int l) {
    return reinterpret_cast<const V*>(T + ((static_cast<int64_t>(x) * nv + y) * nlevels + l) * NN);
  };
  const V a = blk(ua, va, level)[e];
  const V b = blk(ua, vb, level)[e];
  const V c = blk(ub, va, level)[e];
  const V d = blk(ub, vb, level)[e];
  V o;
  const OT q = OT(0.25);
  o.x = ((a.x + b.x) + (c.x + d.x)) * q;
  o.y = ((a.y + b.y) + (c.y + d.y)) * q;
  if constexpr (VEC == 4) {
    o.z = ((a.z + b.z) + (c.z + d.z)) * q;
    o.w = ((a.w + b.w) + (c.w + d.w)) * q;
  }
  reinterpret_cast<V*>(T + (cell * nlevels + level + 1) * NN)[e] = o;
}

__global__ __launch_bounds__(256) void k_range_bruteforce(
    const int32_t* __restrict__ bins, const double* __restrict__ mass, int nu, int nv,
    int nlevels, int N, int K, int64_t nq, const int32_t* __restrict__ q,
    double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  const int P = 2 * K + 1;
  for (int64_t i = wave; i < nq; i += nwaves) {
    const int32_t* r = q + i * 7;
    const int u = glint_wrap(r[0], nu);
    const int v = glint_wrap(r[1], nv);
    const int l = glint_clampi(r[2], 0, nlevels - 1);
    const int slo = glint_clampi(r[3], 0, N), shi = glint_clampi(r[4], 0, N);
    const int tlo = glint_clampi(r[5], 0, N), thi = glint_clampi(r[6], 0, N);
    double acc = 0.0;
    const int k = 1 << l;
    if (slo < shi && tlo < thi) {
      const int h = k >> 1;
      const int64_t kk = static_cast<int64_t>(k) * k;
      for (int64_t t = lane; t < kk; t += 64) {
        const int fi = static_cast<int>(t >> l), fj = static_cast<int>(t & (k - 1));
        int x = (u - h + fi) % nu;
        if (x < 0) x += nu;
        int y = (v - h + fj) % nv;
        if (y < 0) y += nv;
        const int64_t tex = static_cast<int64_t>(x) * nv + y;
        const int is0 = bins[2 * tex] - K, it0 = bins[2 * tex + 1] - K;
        const double* ms = mass + tex * 2 * P;
        const double* mt = ms + P;
        double Ms = 0.0, Mt = 0.0;
        for (int j = 0; j < P; ++j) {
          const int si = is0 + j, ti = it0 + j;
          if (si >= slo && si < shi) Ms += ms[j];
          if (ti >= tlo && ti < thi) Mt += mt[j];
        }
        acc += Ms * Mt;
      }
    }
    acc = glint_wave_sum(acc);
    if (lane == 0) out[i] = acc / (static_cast<double>(k) * k);
  }
}

struct BuildPlan {
  int CB, SR;
  size_t lds;
};

template <typename OT>
bool plan_direct(int level, int NO, int K, int nv, BuildPlan* p) {
  const int k = 1 << level;
  const int P = 2 * K + 1;
  int CB = 16;
  for (; CB >= 1; CB >>= 1) {
    const size_t ntex = static_cast<size_t>(k) * (CB + k - 1);
    const size_t st = glint_round_up(sizeof(int32_t) * 2 * ntex, 16) +
                      glint_round_up(sizeof(OT) * 2 * P * ntex, 16);
    if (st <= kStageBudget) break;
  }
  if (CB < 1) return false;
  if (CB > nv) CB = nv;
  int SR = static_cast<int>(kBlockBudget / (sizeof(OT) * NO));
  if (SR > NO) SR = NO;
  if (SR < 1) return false;
  const size_t ntex = static_cast<size_t>(k) * (CB + k - 1);
  p->CB = CB;
  p->SR = SR;
  p->lds = glint_round_up(sizeof(int32_t) * 2 * ntex, 16) +
           glint_round_up(sizeof(OT) * 2 * P * ntex, 16) + sizeof(OT) * SR * NO;
  return true;
}

template <typename OT>
glint_status build_levels(const glint_ndf_desc* d, const int32_t* bins, const double* mass,
                          OT* T, int direct_levels, int s_off, int t_off, int NO, hipStream_t stream) {
  const int K = glint_window_k(d);
  const int NN = NO * NO;
  for (int l = 0; l < d->nlevels; ++l) {
    BuildPlan p;
    const bool direct = (l < direct_levels) || l == 0;
    if (direct && plan_direct<OT>(l, NO, K, d->nv, &p)) {
      dim3 grid((d->nv + p.CB - 1) / p.CB, d->nu);
      glint_clear_launch_error();
      hipLaunchKernelGGL(k_build_direct<OT>, grid, dim3(kBuildThreads), p.lds, stream, bins,
                         mass, d->nu, d->nv, d->nlevels, K, l, p.CB, p.SR, s_off, t_off, NO, T);
      GLINT_LAUNCHED("k_build_direct");
    } else if (l == 0) {
      return glint_fail(GLINT_E_UNSUPPORTED, "bin window too wide for the direct build");
    } else if (d->nu % (4 << (l - 1)) == 0 && d->nv % (4 << (l - 1)) == 0) {
      // tiles of 8 x 8 output cells where the map allows, else 4 x 4
      const bool m8 = d->nu % (8 << (l - 1)) == 0 && d->nv % (8 << (l - 1)) == 0;
      const int64_t cells = static_cast<int64_t>(d->nu) * d->nv / (m8 ? 64 : 16);
      const int64_t threads = cells * (NN / (16 / static_cast<int>(sizeof(OT))));
      const dim3 grid(static_cast<unsigned>((threads + 255) / 256));
      glint_clear_launch_error();
      if (m8)
        hipLaunchKernelGGL((k_level_double_tile<OT, 8>), grid, dim3(256), 0, stream, T, d->nu, d->nv, d->nlevels, NN,
                           l - 1);
      else
        hipLaunchKernelGGL((k_level_double_tile<OT, 4>), grid, dim3(256), 0, stream, T, d->nu, d->nv, d->nlevels, NN,
                           l - 1);
      GLINT_LAUNCHED("k_level_double_tile");
    } else if (NN <= 1024) {
      const int64_t threads = static_cast<int64_t>(d->nu) * d->nv * (NN / (16 / static_cast<int>(sizeof(OT))));
      glint_clear_launch_error();
      hipLaunchKernelGGL(k_level_double_flat<OT>, dim3(static_cast<unsigned>((threads + 255) / 256)), dim3(256), 0,
                         stream, T, d->nu, d->nv, d->nlevels, NN, l - 1);
      GLINT_LAUNCHED("k_level_double_flat");
    } else {
      dim3 grid(d->nv, d->nu);
      glint_clear_launch_error();
      hipLaunchKernelGGL(k_level_double<OT>, grid, dim3(256), 0, stream, T, d->nu, d->nv,
                         d->nlevels, NO, l - 1);
      GLINT_LAUNCHED("k_level_double");
    }
  }
  return GLINT_OK;
}

size_t bins_bytes(const glint_ndf_desc* d) {
  return glint_round_up(sizeof(int32_t) * 2 * static_cast<size_t>(d->nu) * d->nv, 256);
}

// Scratch of glint_build_tensor_noalloc: the per-texel bin windows and
// masses that glint_build_tensor keeps in its workspace, in a file-scope
// device array instead (each device holds its own copy while the library is
// loaded).  Host code never passes `scratch` itself to a kernel: on the host
// the name is a stand-in, not a device address.  The device address comes
// from hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kNoAllocScratchBytes = GLINT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_addr[kMaxDevices] = {};

glint_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return glint_fail(GLINT_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return glint_fail(GLINT_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_addr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return glint_fail(GLINT_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return GLINT_OK;
}

}  // namespace

glint_status glint_build_window(const glint_ndf_desc* desc, const int32_t* bins, const double* mass, void* T,
                                glint_dtype T_dtype, int32_t direct_levels, int32_t s_off, int32_t t_off,
                                int32_t nout, hipStream_t stream) {
  GLINT_REQUIRE(nout >= 1 && s_off >= 0 && t_off >= 0 && s_off + nout <= desc->nbins && t_off + nout <= desc->nbins,
                "bin window [%d, %d) x [%d, %d) outside the %d bins", s_off, s_off + nout, t_off, t_off + nout,
                desc->nbins);
  GLINT_REQUIRE(nout * nout % 4 == 0, "bin window of %d x %d bins: the level doubling moves 16-byte words", nout,
                nout);
  if (direct_levels <= 0) direct_levels = 3;
  if (T_dtype == GLINT_F64)
    return build_levels<double>(desc, bins, mass, static_cast<double*>(T), direct_levels, s_off, t_off, nout,
                                stream);
  GLINT_SUPPORT(T_dtype == GLINT_F32, "T dtype must be F64 or F32");
  return build_levels<float>(desc, bins, mass, static_cast<float*>(T), direct_levels, s_off, t_off, nout, stream);
}

extern "C" {

glint_status glint_texel_bins(const glint_ndf_desc* desc, const float* nxy, int32_t* bins,
                              double* mass, hipStream_t stream) {
  glint_status st = glint_check_desc(desc);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(nxy && bins && mass, "null pointer argument");
  const int64_t n2 = 2 * static_cast<int64_t>(desc->nu) * desc->nv;
  const int K = glint_window_k(desc);
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_texel_bins, dim3(static_cast<unsigned>((n2 + 255) / 256)), dim3(256), 0,
                     stream, nxy, n2, desc->nbins, desc->sigma, K, bins, mass);
  GLINT_LAUNCHED("k_texel_bins");
  return GLINT_OK;
}

size_t glint_build_tensor_workspace(const glint_ndf_desc* desc) {
  if (glint_check_desc(desc) != GLINT_OK) return 0;
  const int K = glint_window_k(desc);
  return bins_bytes(desc) +
         glint_round_up(sizeof(double) * 2 * static_cast<size_t>(desc->nu) * desc->nv * (2 * K + 1), 256);
}

glint_status glint_build_tensor(const glint_ndf_desc* desc, const float* nxy, void* T,
                                glint_dtype T_dtype, int32_t direct_levels, void* workspace,
                                size_t workspace_bytes, hipStream_t stream) {
  glint_status st = glint_check_desc(desc);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(nxy && T && workspace, "null pointer argument");
  GLINT_REQUIRE(glint_aligned(T, 16) && glint_aligned(workspace, 16), "T and workspace must be 16-byte aligned");
  GLINT_SUPPORT(T_dtype == GLINT_F64 || T_dtype == GLINT_F32, "T dtype must be F64 or F32");
  const size_t need = glint_build_tensor_workspace(desc);
  if (workspace_bytes < need)
    return glint_fail(GLINT_E_WORKSPACE, "workspace %zu < %zu bytes", workspace_bytes, need);
  if (direct_levels <= 0) direct_levels = 3;
  int32_t* bins = static_cast<int32_t*>(workspace);
  double* mass = reinterpret_cast<double*>(static_cast<unsigned char*>(workspace) + bins_bytes(desc));
  st = glint_texel_bins(desc, nxy, bins, mass, stream);
  if (st != GLINT_OK) return st;
  if (T_dtype == GLINT_F64)
    return build_levels<double>(desc, bins, mass, static_cast<double*>(T), direct_levels, 0, 0, desc->nbins,
                                stream);
  return build_levels<float>(desc, bins, mass, static_cast<float*>(T), direct_levels, 0, 0, desc->nbins, stream);
}

glint_status glint_build_tensor_noalloc(const glint_ndf_desc* desc, const float* nxy, void* T,
                                        glint_dtype T_dtype, int32_t direct_levels, hipStream_t stream) {
  glint_status st = glint_check_desc(desc);
  if (st != GLINT_OK) return st;
  const size_t need = glint_build_tensor_workspace(desc);
  if (need > kNoAllocScratchBytes)
    return glint_fail(GLINT_E_UNSUPPORTED, "the map needs %zu bytes of scratch, the no-allocation build has %zu",
                      need, kNoAllocScratchBytes);
  void* ws = nullptr;
  if ((st = scratch_address(&ws)) != GLINT_OK) return st;
  return glint_build_tensor(desc, nxy, T, T_dtype, direct_levels, ws, kNoAllocScratchBytes, stream);
}

glint_status glint_range_bruteforce(const glint_ndf_desc* desc, const int32_t* bins,
                                    const double* mass, int64_t nq, const int32_t* q,
                                    double* out, hipStream_t stream) {
  glint_status st = glint_check_desc(desc);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(nq >= 0, "nq must be >= 0");
  if (nq == 0) return GLINT_OK;
  GLINT_REQUIRE(bins && mass && q && out, "null pointer argument");
  const int K = glint_window_k(desc);
  const int64_t waves = nq < (int64_t(1) << 20) ? nq : (int64_t(1) << 20);
  const unsigned blocks = static_cast<unsigned>((waves + 3) / 4);
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_range_bruteforce, dim3(blocks), dim3(256), 0, stream, bins, mass,
                     desc->nu, desc->nv, desc->nlevels, desc->nbins, K, nq, q, out);
  GLINT_LAUNCHED("k_range_bruteforce");
  return GLINT_OK;
}

}  // extern "C"
