// The clustered layout of the compression (Sec. 4.2, Eq. compress and its
// practical choices): every NDF image is cut into t x t angular blocks and
// the footprints are grouped by the cs x cs texel region of their centre;
// the blocks of one region and one angular position form a 3-way tensor
// D[a][b][f] (f = (du cs + dv) nl + l) that gets its own rank-R CP.  The
// range query (Sec. 4.4) splits a box at block edges and adds the
// block-local queries.
//
// CP-ALS kernel: one 256-thread workgroup per (region, block) tensor runs
// every sweep with its factors, Grams and the (a,b)-by-rank product
// P = D x_f Z resident in LDS in FP64; D is streamed from the tensor T each
// sweep (two passes: P for the X and Y updates, then D against the
// Khatri-Rao product of X and Y for Z).
#include <cstdint>

#include "common.h"

namespace {

constexpr double kBlankRtol = 1e-12;    // blank block: sum |D| <= kBlankRtol * L
constexpr double kPivotRtol = 1e-13;    // Cholesky breakdown
constexpr double kRidgeRtol = 1e-10;    // normal equations use G + mu I, mu = kRidgeRtol * trace(G) / R
constexpr int kClThreads = 256;
// footprints per staged chunk of the Z pass (64 bytes per angular bin)
template <typename TT>
constexpr int stage_footprints() { return 64 / static_cast<int>(sizeof(TT)); }

// SplitMix64 (Steele, Lea and Flood) as a counter-based generator: the
// (counter+1)-th output of the generator seeded with `seed`, as U[0, 1).
__device__ __forceinline__ double sm64_uniform(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return static_cast<double>(z >> 11) * (1.0 / 9007199254740992.0);
}

struct ClusterArgs {
  const void* T;
  int nu, nv, nl, N;
  int t, cs, ncv, nb, L;
  int iters;
  uint64_t seed;
  float* X;
  float* Y;
  float* Z;
  uint8_t* blank;
  int* info;
};

// Offsets of the LDS arrays (doubles) of the ALS kernel.
struct ClusterLds {
  int x, y, z, p, gx, gy, gz, gm, lam, red, mtmp, stage, total_doubles;
};

__host__ __device__ inline ClusterLds cluster_lds(int t, int L, int R, int stage_elt_bytes) {
  ClusterLds o;
  int at = 0;
  auto take = [&](int n) {
    const int a = at;
    at += (n + 1) / 2 * 2;   // keep 16-byte alignment
    return a;
  };
  o.x = take(t * R);
  o.y = take(t * R);
  o.z = take(L * R);
  o.p = take(t * t * R);
  o.gx = take(R * R);
  o.gy = take(R * R);
  o.gz = take(R * R);
  o.gm = take(R * R);
  o.lam = take(R);
  o.red = take(kClThreads);
  o.mtmp = take(t * R);
  o.stage = take((64 / stage_elt_bytes * t * t * stage_elt_bytes + 7) / 8);
  o.total_doubles = at;
  return o;
}

template <typename TT>
struct TensorView {
  const TT* T;
  int64_t cell0;       // cell index of footprint f = 0
  int nv, nl, cs, N;
  __device__ int64_t ab_off(int a, int b, int zs, int zt, int t) const {
    return static_cast<int64_t>(zs * t + a) * N + zt * t + b;
  }
  // element (a, b) of footprint f, at offset ab (from ab_off)
  __device__ __forceinline__ double at(int64_t ab, int f) const {
    const int du = f / (cs * nl), dv = (f / nl) % cs, l = f % nl;
    const int64_t cell = cell0 + (static_cast<int64_t>(du) * nv + dv) * nl + l;
    return static_cast<double>(T[cell * N * N + ab]);
  }
};

// A = M (G + mu I)^-1 row by row for `rows` rows held in LDS (in place),
// with Gm holding the Cholesky factor (lower, row-major, R x R).
template <int R>
__device__ void solve_rows(double* Mrows, int rows, const double* Lc) {
  for (int row = threadIdx.x; row < rows; row += blockDim.x) {
    double* m = Mrows + row * R;
    double y[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      double s = m[k];
      for (int i = 0; i < k; ++i) s -= Lc[k * R + i] * y[i];
      y[k] = s / Lc[k * R + k];
    }
#pragma unroll
    for (int k = R - 1; k >= 0; --k) {
      double s = y[k];
      for (int i = k + 1; i < R; ++i) s -= Lc[i * R + k] * m[i];
      m[k] = s / Lc[k * R + k];
    }
  }
}

// Gm = G1 o G2 + mu I factored in place (lower Cholesky); returns false on
// breakdown (the same for every thread).
template <int R>
__device__ bool cholesky_hadamard(const double* G1, const double* G2, double* Gm, double* red) {
  for (int i = threadIdx.x; i < R * R; i += blockDim.x) Gm[i] = G1[i] * G2[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0.0;
    for (int k = 0; k < R; ++k) tr += Gm[k * R + k];
    const double mu = kRidgeRtol * tr / R;
    for (int k = 0; k < R; ++k) Gm[k * R + k] += mu;
  }
  __syncthreads();
  // diagonal entries of G + mu I for the breakdown rule
  if (threadIdx.x < R) red[threadIdx.x] = Gm[threadIdx.x * R + threadIdx.x];
  __syncthreads();
  bool ok = true;
  for (int j = 0; j < R; ++j) {
    // pivot (every thread computes it from the same LDS values)
    double d = Gm[j * R + j];
    for (int k = 0; k < j; ++k) d -= Gm[j * R + k] * Gm[j * R + k];
    if (!(d > kPivotRtol * red[j])) {
      ok = false;
      break;
    }
    const double ljj = sqrt(d);
    __syncthreads();
    if (threadIdx.x == 0) Gm[j * R + j] = ljj;
    for (int i = j + 1 + static_cast<int>(threadIdx.x); i < R; i += blockDim.x) {
      double s = Gm[i * R + j];
      for (int k = 0; k < j; ++k) s -= Gm[i * R + k] * Gm[j * R + k];
      Gm[i * R + j] = s / ljj;
    }
    __syncthreads();
  }
  __syncthreads();
  return ok;
}

// G = F^T F for F [rows][R] in LDS.
template <int R>
__device__ void gram_lds(const double* F, int rows, double* G) {
  for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) {
    const int i = idx / R, j = idx % R;
    double s = 0.0;
    for (int row = 0; row < rows; ++row) s += F[row * R + i] * F[row * R + j];
    G[idx] = s;
  }
  __syncthreads();
}

// unit columns; lam[r] = column norm (zero columns stay zero)
template <int R>
__device__ void normalize_cols(double* F, int rows, double* lam) {
  if (threadIdx.x < R) {
    double s = 0.0;
    for (int row = 0; row < rows; ++row) s += F[row * R + threadIdx.x] * F[row * R + threadIdx.x];
    lam[threadIdx.x] = sqrt(s);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < rows * R; idx += blockDim.x) {
    const double n = lam[idx % R];
    if (n > 0.0) F[idx] /= n;
  }
  __syncthreads();
}

template <typename TT, int R>
__global__ __launch_bounds__(kClThreads) void k_cluster_als(ClusterArgs c) {
  extern __shared__ __align__(16) double cl_lds[];
  const int t = c.t, L = c.L, tt = t * t;
  const ClusterLds o = cluster_lds(t, L, R, sizeof(TT));
  double* X = cl_lds + o.x;
  double* Y = cl_lds + o.y;
  double* Z = cl_lds + o.z;
  double* P = cl_lds + o.p;
  double* GX = cl_lds + o.gx;
  double* GY = cl_lds + o.gy;
  double* GZ = cl_lds + o.gz;
  double* Gm = cl_lds + o.gm;
  double* lam = cl_lds + o.lam;
  double* red = cl_lds + o.red;
  double* Mt = cl_lds + o.mtmp;
  TT* stage = reinterpret_cast<TT*>(cl_lds + o.stage);

  const int tensor = blockIdx.x;
  const int zt = tensor % c.nb, zs = (tensor / c.nb) % c.nb;
  const int cv = (tensor / (c.nb * c.nb)) % c.ncv, cu = tensor / (c.nb * c.nb * c.ncv);
  TensorView<TT> D;
  D.T = static_cast<const TT*>(c.T);
  D.cell0 = (static_cast<int64_t>(cu * c.cs) * c.nv + cv * c.cs) * c.nl;
  D.nv = c.nv; D.nl = c.nl; D.cs = c.cs; D.N = c.N;
  const int my_ab = threadIdx.x;
  const bool ab_active = my_ab < tt;
  const int64_t ab_off = ab_active ? D.ab_off(my_ab / t, my_ab % t, zs, zt, t) : 0;

  // blank check: sum |D|
  {
    double s = 0.0;
    if (ab_active)
      for (int f = 0; f < L; ++f) s += fabs(D.at(ab_off, f));
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kClThreads / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    const bool blank = !(red[0] > kBlankRtol * L);
    __syncthreads();
    if (blank) {
      for (int i = threadIdx.x; i < t * R; i += blockDim.x) {
        c.X[static_cast<int64_t>(tensor) * t * R + i] = 0.0f;
        c.Y[static_cast<int64_t>(tensor) * t * R + i] = 0.0f;
      }
      for (int i = threadIdx.x; i < L * R; i += blockDim.x) c.Z[static_cast<int64_t>(tensor) * L * R + i] = 0.0f;
      if (threadIdx.x == 0) {
        c.blank[tensor] = 1;
        atomicAdd(&c.info[1], 1);
      }
      return;
    }
  }

  // initial factors (SplitMix64 counters) and Grams; lambda = 1
  const uint64_t rows_max = t > L ? t : L;
  for (int i = threadIdx.x; i < t * R; i += blockDim.x) {
    const uint64_t row = i / R, r = i % R;
    X[i] = sm64_uniform(c.seed, ((static_cast<uint64_t>(tensor) * 3 + 0) * rows_max + row) * R + r);
    Y[i] = sm64_uniform(c.seed, ((static_cast<uint64_t>(tensor) * 3 + 1) * rows_max + row) * R + r);
  }
  for (int i = threadIdx.x; i < L * R; i += blockDim.x) {
    const uint64_t row = i / R, r = i % R;
    Z[i] = sm64_uniform(c.seed, ((static_cast<uint64_t>(tensor) * 3 + 2) * rows_max + row) * R + r);
  }
  if (threadIdx.x < R) lam[threadIdx.x] = 1.0;
  __syncthreads();
  gram_lds<R>(X, t, GX);
  gram_lds<R>(Y, t, GY);
  gram_lds<R>(Z, L, GZ);
  int fails = 0;

  for (int it = 0; it < c.iters; ++it) {
    // pass A: P[ab][r] = sum_f D[ab][f] Z[f][r]
    if (ab_active) {
      double acc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = 0.0;
      for (int f = 0; f < L; ++f) {
        const double d = D.at(ab_off, f);
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] += d * Z[f * R + r];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) P[my_ab * R + r] = acc[r];
    }
    __syncthreads();
    // mode X: M[a][r] = sum_b P[ab][r] Y[b][r]
    for (int idx = threadIdx.x; idx < t * R; idx += blockDim.x) {
      const int a = idx / R, r = idx % R;
      double s = 0.0;
      for (int b = 0; b < t; ++b) s += P[(a * t + b) * R + r] * Y[b * R + r];
      Mt[idx] = s;
    }
    __syncthreads();
    if (cholesky_hadamard<R>(GY, GZ, Gm, red)) {
      solve_rows<R>(Mt, t, Gm);
      __syncthreads();
      for (int i = threadIdx.x; i < t * R; i += blockDim.x) X[i] = Mt[i];
      __syncthreads();
      normalize_cols<R>(X, t, lam);
      gram_lds<R>(X, t, GX);
    } else {
      ++fails;
    }
    // mode Y: M[b][r] = sum_a P[ab][r] X[a][r]
    for (int idx = threadIdx.x; idx < t * R; idx += blockDim.x) {
      const int b = idx / R, r = idx % R;
      double s = 0.0;
      for (int a = 0; a < t; ++a) s += P[(a * t + b) * R + r] * X[a * R + r];
      Mt[idx] = s;
    }
    __syncthreads();
    if (cholesky_hadamard<R>(GX, GZ, Gm, red)) {
      solve_rows<R>(Mt, t, Gm);
      __syncthreads();
      for (int i = threadIdx.x; i < t * R; i += blockDim.x) Y[i] = Mt[i];
      __syncthreads();
      normalize_cols<R>(Y, t, lam);
      gram_lds<R>(Y, t, GY);
    } else {
      ++fails;
    }
    // mode Z (factored first: Z is overwritten in place only when it succeeds)
    if (cholesky_hadamard<R>(GX, GY, Gm, red)) {
      for (int idx = threadIdx.x; idx < tt * R; idx += blockDim.x) {
        const int ab = idx / R, r = idx % R;
        P[idx] = X[(ab / t) * R + r] * Y[(ab % t) * R + r];      // Khatri-Rao of X and Y
      }
      __syncthreads();
      constexpr int FC = stage_footprints<TT>();
      for (int f0 = 0; f0 < L; f0 += FC) {
        const int nf = L - f0 < FC ? L - f0 : FC;
        if (ab_active)
          for (int i = 0; i < nf; ++i) stage[i * tt + my_ab] = static_cast<TT>(D.at(ab_off, f0 + i));
        __syncthreads();
        for (int idx = threadIdx.x; idx < nf * R; idx += blockDim.x) {
          const int i = idx / R, r = idx % R;
          double s = 0.0;
          for (int ab = 0; ab < tt; ++ab) s += static_cast<double>(stage[i * tt + ab]) * P[ab * R + r];
          Z[(f0 + i) * R + r] = s;
        }
        __syncthreads();
      }
      solve_rows<R>(Z, L, Gm);
      __syncthreads();
      normalize_cols<R>(Z, L, lam);
      gram_lds<R>(Z, L, GZ);
    } else {
      ++fails;
    }
  }
  // outputs: X, Y, Z * lambda (FP32)
  for (int i = threadIdx.x; i < t * R; i += blockDim.x) {
    c.X[static_cast<int64_t>(tensor) * t * R + i] = static_cast<float>(X[i]);
    c.Y[static_cast<int64_t>(tensor) * t * R + i] = static_cast<float>(Y[i]);
  }
  for (int i = threadIdx.x; i < L * R; i += blockDim.x)
    c.Z[static_cast<int64_t>(tensor) * L * R + i] = static_cast<float>(Z[i] * lam[i % R]);
  if (threadIdx.x == 0) {
    c.blank[tensor] = 0;
    if (fails) atomicAdd(&c.info[0], fails);
  }
}

__global__ void k_cluster_info_init(int* info) {
  if (threadIdx.x < 2) info[threadIdx.x] = 0;
}

// C[b][j][r] = sum_{s<j} S[b][s][r] (FP64 accumulation), FP32 out.
__global__ void k_cumulative_batched(int64_t nbatch, int n, int R, const float* __restrict__ S,
                                     float* __restrict__ C) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= nbatch * R) return;
  const int64_t b = idx / R;
  const int r = static_cast<int>(idx % R);
  const float* s = S + b * n * R + r;
  float* cc = C + b * (n + 1) * R + r;
  double acc = 0.0;
  cc[0] = 0.0f;
  for (int j = 0; j < n; ++j) {
    acc += static_cast<double>(s[static_cast<int64_t>(j) * R]);
    cc[static_cast<int64_t>(j + 1) * R] = static_cast<float>(acc);
  }
}

// ---------------------------------------------------------------------------
// block-split range query on the clustered tables
// ---------------------------------------------------------------------------

struct ClQueryArgs {
  const float* CX;   // [ntensor][t+1][R]
  const float* CY;
  const float* Z;    // [ntensor][L][R]
  int t, cs, nu, nv, nl, N, ncv, nb, L;
  int64_t nq;
  const int32_t* q;
  float* out;
};

struct alignas(16) ClRec {
  int tensor0;   // tensor index of block (0, 0) of the region
  int f;
  int slo, shi, tlo, thi;
  int pad0, pad1;
};

constexpr int kClQueryThreads = 256;

// lane group of LPQ = R / 4 lanes per query, 4 ranks (16 bytes) per lane
template <int R>
__global__ __launch_bounds__(kClQueryThreads) void k_query_clustered(ClQueryArgs a) {
  constexpr int RPL = R < 4 ? R : 4;
  constexpr int LPQ = R / RPL;
  __shared__ ClRec recs[kClQueryThreads / 64][64];
  const int lane = threadIdx.x & 63;
  const int g = lane / LPQ, j = lane % LPQ, r0 = j * RPL;
  ClRec* wr = recs[threadIdx.x >> 6];
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  const int t = a.t;
  for (int64_t base = wave * 64; base < a.nq; base += nwaves * 64) {
    {
      const int64_t qi = base + lane;
      const int64_t qc = qi < a.nq ? qi : a.nq - 1;
      const int32_t* rec = a.q + qc * 7;
      const int u = glint_wrap(rec[0], a.nu), v = glint_wrap(rec[1], a.nv);
      const int l = glint_clampi(rec[2], 0, a.nl - 1);
      ClRec cr;
      cr.tensor0 = ((u / a.cs) * a.ncv + v / a.cs) * a.nb * a.nb;
      cr.f = ((u % a.cs) * a.cs + v % a.cs) * a.nl + l;
      cr.slo = glint_clampi(rec[3], 0, a.N);
      cr.shi = glint_clampi(rec[4], 0, a.N);
      cr.tlo = glint_clampi(rec[5], 0, a.N);
      cr.thi = glint_clampi(rec[6], 0, a.N);
      cr.pad0 = cr.pad1 = 0;
      wr[lane] = cr;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    float res = 0.0f;
    for (int jj = 0; jj < LPQ; ++jj) {
      const ClRec cr = wr[g * LPQ + jj];
      float acc = 0.0f;
      if (cr.slo < cr.shi && cr.tlo < cr.thi) {
        for (int zs = cr.slo / t; zs <= (cr.shi - 1) / t; ++zs) {
          const int a0 = max(cr.slo, zs * t) - zs * t, a1 = min(cr.shi, (zs + 1) * t) - zs * t;
          for (int zt = cr.tlo / t; zt <= (cr.thi - 1) / t; ++zt) {
            const int b0 = max(cr.tlo, zt * t) - zt * t, b1 = min(cr.thi, (zt + 1) * t) - zt * t;
            const int64_t tensor = cr.tensor0 + zs * a.nb + zt;
            const float* cx = a.CX + tensor * (t + 1) * R + r0;
            const float* cy = a.CY + tensor * (t + 1) * R + r0;
            const float* z = a.Z + (tensor * a.L + cr.f) * R + r0;
#pragma unroll
            for (int e = 0; e < RPL; ++e)
              acc += z[e] * (cx[a1 * R + e] - cx[a0 * R + e]) * (cy[b1 * R + e] - cy[b0 * R + e]);
          }
        }
      }
      acc = glint_group_sum<LPQ>(acc);
      res = (j == jj) ? acc : res;
    }
    __builtin_amdgcn_wave_barrier();
    const int64_t qo = base + g * LPQ + j;
    if (qo < a.nq) a.out[qo] = res;
  }
}

int g_cl_cus = 0, g_cl_lds = 0;

glint_status cl_device() {
  if (g_cl_cus > 0) return GLINT_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&g_cl_cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&g_cl_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return glint_fail(GLINT_E_HIP, "hipDeviceGetAttribute failed");
  return GLINT_OK;
}

struct ClShape {
  int t, ncu, ncv, nb, L;
  int64_t ntensor;
};

glint_status cluster_shape(const glint_ndf_desc* d, const glint_cluster_desc* cd, ClShape* s) {
  glint_status st = glint_check_desc(d);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(cd != nullptr, "cluster desc is NULL");
  GLINT_REQUIRE(cd->t >= 1 && cd->cs >= 1, "block side and region side must be positive");
  s->t = cd->t < d->nbins ? cd->t : d->nbins;
  GLINT_REQUIRE(d->nbins % s->t == 0, "block side %d must divide nbins %d", s->t, d->nbins);
  GLINT_SUPPORT(s->t <= 16, "block side %d above 16", s->t);
  GLINT_REQUIRE(d->nu % cd->cs == 0 && d->nv % cd->cs == 0, "region side %d must divide the map sides", cd->cs);
  GLINT_SUPPORT(cd->R == 4 || cd->R == 8 || cd->R == 16 || cd->R == 32, "rank %d not in {4,8,16,32}", cd->R);
  s->ncu = d->nu / cd->cs;
  s->ncv = d->nv / cd->cs;
  s->nb = d->nbins / s->t;
  s->L = cd->cs * cd->cs * d->nlevels;
  s->ntensor = static_cast<int64_t>(s->ncu) * s->ncv * s->nb * s->nb;
  GLINT_SUPPORT(s->ntensor < (int64_t{1} << 31), "too many region-and-block tensors");
  return GLINT_OK;
}

template <typename TT, int R>
glint_status launch_cluster_als(const ClusterArgs& c, hipStream_t stream) {
  const ClusterLds o = cluster_lds(c.t, c.L, R, sizeof(TT));
  const size_t lds = sizeof(double) * o.total_doubles;
  if (static_cast<int>(lds) > g_cl_lds)
    return glint_fail(GLINT_E_UNSUPPORTED, "clustered ALS needs %zu bytes of LDS (device max %d)", lds, g_cl_lds);
  const int64_t ntensor = static_cast<int64_t>(c.ncv) * (c.nu / c.cs) * c.nb * c.nb;
  hipLaunchKernelGGL((k_cluster_als<TT, R>), dim3(static_cast<unsigned>(ntensor)), dim3(kClThreads), lds, stream, c);
  GLINT_LAUNCHED("k_cluster_als");
  return GLINT_OK;
}

}  // namespace

extern "C" {

glint_status glint_cp_als_clustered(const glint_ndf_desc* desc, const glint_cluster_desc* cd, const void* T,
                                    glint_dtype T_dtype, int32_t iters, uint64_t seed, float* X, float* Y,
                                    float* Z, uint8_t* blank, int32_t* info, hipStream_t stream) {
  ClShape s;
  glint_status st = cluster_shape(desc, cd, &s);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(T && X && Y && Z && blank && info, "null pointer argument");
  GLINT_REQUIRE(iters >= 1, "iters must be >= 1");
  GLINT_SUPPORT(T_dtype == GLINT_F32 || T_dtype == GLINT_F64, "T must be F32 or F64");
  if ((st = cl_device()) != GLINT_OK) return st;
  ClusterArgs c;
  c.T = T; c.nu = desc->nu; c.nv = desc->nv; c.nl = desc->nlevels; c.N = desc->nbins;
  c.t = s.t; c.cs = cd->cs; c.ncv = s.ncv; c.nb = s.nb; c.L = s.L;
  c.iters = iters; c.seed = seed; c.X = X; c.Y = Y; c.Z = Z; c.blank = blank; c.info = info;
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_cluster_info_init, dim3(1), dim3(64), 0, stream, info);
  GLINT_LAUNCHED("k_cluster_info_init");
  const bool f64 = T_dtype == GLINT_F64;
  switch (cd->R) {
    case 4: return f64 ? launch_cluster_als<double, 4>(c, stream) : launch_cluster_als<float, 4>(c, stream);
    case 8: return f64 ? launch_cluster_als<double, 8>(c, stream) : launch_cluster_als<float, 8>(c, stream);
    case 16: return f64 ? launch_cluster_als<double, 16>(c, stream) : launch_cluster_als<float, 16>(c, stream);
    default: return f64 ? launch_cluster_als<double, 32>(c, stream) : launch_cluster_als<float, 32>(c, stream);
  }
}

glint_status glint_make_cumulative_batched(int64_t nbatch, int32_t n, int32_t R, const float* S, float* C,
                                           hipStream_t stream) {
  GLINT_REQUIRE(nbatch >= 0 && n >= 1 && R >= 1, "bad sizes");
  if (nbatch == 0) return GLINT_OK;
  GLINT_REQUIRE(S && C, "null pointer argument");
  const int64_t threads = nbatch * R;
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_cumulative_batched, dim3(static_cast<unsigned>((threads + 255) / 256)), dim3(256), 0,
                     stream, nbatch, n, R, S, C);
  GLINT_LAUNCHED("k_cumulative_batched");
  return GLINT_OK;
}

glint_status glint_query_clustered(const glint_clustered* f, int64_t nq, const int32_t* q, float* out,
                                   hipStream_t stream) {
  GLINT_REQUIRE(f != nullptr, "tables are NULL");
  glint_ndf_desc d;
  d.nu = f->nu; d.nv = f->nv; d.nlevels = f->nl; d.nbins = f->nbins; d.sigma = 0.01;
  glint_cluster_desc cd;
  cd.t = f->t; cd.cs = f->cs; cd.R = f->R;
  ClShape s;
  glint_status st = cluster_shape(&d, &cd, &s);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(f->t == s.t, "block side must be min(t, nbins) = %d", s.t);
  GLINT_REQUIRE(nq >= 0, "nq must be >= 0");
  if (nq == 0) return GLINT_OK;
  GLINT_REQUIRE(f->CX && f->CY && f->Z && q && out, "null pointer argument");
  GLINT_REQUIRE(glint_aligned(f->CX, 16) && glint_aligned(f->CY, 16) && glint_aligned(f->Z, 16),
                "tables must be 16-byte aligned");
  if ((st = cl_device()) != GLINT_OK) return st;
  ClQueryArgs a;
  a.CX = f->CX; a.CY = f->CY; a.Z = f->Z;
  a.t = s.t; a.cs = f->cs; a.nu = f->nu; a.nv = f->nv; a.nl = f->nl; a.N = f->nbins;
  a.ncv = s.ncv; a.nb = s.nb; a.L = s.L; a.nq = nq; a.q = q; a.out = out;
  const int64_t waves = (nq + 63) / 64;
  int64_t blocks = (waves + 3) / 4;
  const int64_t cap = static_cast<int64_t>(g_cl_cus) * 8;
  if (blocks > cap) blocks = cap;
  glint_clear_launch_error();
  switch (f->R) {
    case 4: hipLaunchKernelGGL(k_query_clustered<4>, dim3(blocks), dim3(kClQueryThreads), 0, stream, a); break;
    case 8: hipLaunchKernelGGL(k_query_clustered<8>, dim3(blocks), dim3(kClQueryThreads), 0, stream, a); break;
    case 16: hipLaunchKernelGGL(k_query_clustered<16>, dim3(blocks), dim3(kClQueryThreads), 0, stream, a); break;
    default: hipLaunchKernelGGL(k_query_clustered<32>, dim3(blocks), dim3(kClQueryThreads), 0, stream, a); break;
  }
  GLINT_LAUNCHED("k_query_clustered");
  return GLINT_OK;
}

}  // extern "C"
