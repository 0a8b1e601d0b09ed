// The clustered layout of the compression (Sec. 4.2, Eq. compress and its
// practical choices): every NDF image is cut into t x t angular blocks and
// the footprints are grouped by the cs x cs texel region of their centre;
// the blocks of one region and one angular position form a 3-way tensor
// D[a][b][f] (f = (du cs + dv) nl + l) that gets its own rank-R CP.  The
// range query (Sec. 4.4) splits a box at block edges and adds the
// block-local queries.
//
// CP-ALS: a high-occupancy pre-pass flags the blank image blocks (Sec. 4.2:
// only the L' non-empty blocks of a cluster are stacked); then one 512-thread
// workgroup per block tensor stacks the rest and runs every sweep with its
// factors, Grams and the
// (a,b)-by-rank product P = D x_f Z resident in LDS in FP64.  D is streamed
// from the tensor T twice per sweep, and both streams are dense
// contractions on the matrix cores (v_mfma_f64_16x16x4f64):
//   pass A  P[ab][r] = sum_f D[ab][f] Z[f][r]          (for the X and Y updates)
//   pass B  Z[f][r]  = sum_ab D[ab][f] X[a][r] Y[b][r]  (the Z update)
// Pass A reads D straight from HBM (16 consecutive bins of one footprint per
// lane group, double-buffered); pass B stages D through a padded LDS tile so
// that each wave owns 16 footprints of the output.  The Grams are MFMA
// products too, and the column norms come from their diagonals.
#include <cstdint>

#include "common.h"

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr double kBlankTol = 1e-12;     // blank image block: sum of |values| <= kBlankTol
constexpr double kPivotRtol = 1e-13;    // Cholesky breakdown
constexpr double kRidgeRtol = 1e-10;    // normal equations use G + mu I, mu = kRidgeRtol * trace(G) / R
constexpr int kClThreads = 512;
constexpr int kClWaves = kClThreads / 64;
constexpr int kFR = 16 * kClWaves;      // footprints per pass-B range: 16 per wave
// pass-A MFMA steps (4 footprints each) per prefetched batch: one batch
// in flight while the previous one runs on the matrix cores
template <typename TT>
constexpr int pass_a_batch() { return sizeof(TT) == 4 ? 8 : 8; }

// pass-B stage: kFR footprints x AB bins of T, rows padded so that the 16
// footprints x 4 bins an MFMA operand read touches fall in distinct banks
template <typename TT>
constexpr int stage_ab() { return sizeof(TT) == 4 ? 64 : 32; }
template <typename TT>
constexpr int stage_stride() { return stage_ab<TT>() + (sizeof(TT) == 4 ? 4 : 2); }   // 272 bytes
constexpr int kGramPart = 2048;         // doubles of per-wave Gram partials (reuse the stage)

// v_mfma_f64_16x16x4f64: A[i][k] from lane i + 16k, B[k][j] from lane j + 16k;
// D[i][j] in lane j + 16 (i % 4), item i / 4.
__device__ __forceinline__ f64x4 mfma64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

struct ClusterArgs {
  const void* T;
  int nu, nv, nl, N;
  int t, cs, ncv, nb, L;
  int iters;
  int ntensor;
  int R;
  uint64_t seed;
  float* X;
  float* Y;
  float* Z;
  uint8_t* blank;
  int* info;
  // tensor i of T is the layout's tensor i * tmul + tadd (T holding one
  // angular block: tmul = nb^2 of the whole image, tadd = its zs nb + zt)
  int64_t tmul, tadd;
  // compact layout (null: dense Z [ntensor][L][R] with zero blank rows):
  // zidx[tensor][f] is the footprint's row of Z or -1 (blank); the mass
  // pass writes 0/1 flags there and counts[tensor] the non-blank footprints
  int32_t* zidx;
  int32_t* counts;
  // Z factors in global memory (one slot of zws_stride doubles per
  // workgroup) where the LDS cannot hold them
  double* zws;
  int64_t zws_stride;
};

// Offsets of the LDS arrays (in doubles) of the ALS kernel.  Z rows are
// padded to R + 1 doubles (the per-row solves then spread over the banks).
struct ClusterLds {
  int x, y, mt, z, p, gx, gy, gz, gm, lam, dg, dl, foff, keep, rowof, stage, total_doubles;
};

__host__ __device__ inline ClusterLds cluster_lds(int t, int L, int R, int stage_doubles, bool z_global) {
  ClusterLds o;
  int at = 0;
  auto take = [&](int n) {
    const int a = at;
    at += (n + 1) / 2 * 2;   // keep 16-byte alignment
    return a;
  };
  o.x = take(t * R);
  o.y = take(t * R);
  o.mt = take(t * R);
  o.z = z_global ? -1 : take(L * (R + 1));
  o.p = take(t * t * R);
  o.gx = take(R * R);
  o.gy = take(R * R);
  o.gz = take(R * R);
  o.gm = take(R * R);
  o.lam = take(R);
  o.dg = take(R);
  o.dl = take(R);
  o.foff = take(L);            // int64 footprint offsets of the stacked rows
  o.keep = take((L + 1) / 2);  // int: footprint of stacked row j
  o.rowof = take((L + 1) / 2); // int: stacked row of footprint f, or -1 (blank)
  o.stage = take(stage_doubles > kGramPart ? stage_doubles : kGramPart);
  o.total_doubles = at;
  return o;
}

template <typename TT>
__host__ __device__ constexpr int stage_doubles() {
  return (kFR * stage_stride<TT>() * static_cast<int>(sizeof(TT)) + 7) / 8;
}

// Position of one block tensor inside T.
struct BlockPos {
  int64_t base;   // element offset of footprint f = 0, bin (zs t, zt t)
  int zs, zt;
};

__device__ __forceinline__ BlockPos block_pos(const ClusterArgs& c, int tensor) {
  BlockPos b;
  b.zt = tensor % c.nb;
  b.zs = (tensor / c.nb) % c.nb;
  const int cv = (tensor / (c.nb * c.nb)) % c.ncv, cu = tensor / (c.nb * c.nb * c.ncv);
  const int64_t cell0 = (static_cast<int64_t>(cu) * c.cs * c.nv + static_cast<int64_t>(cv) * c.cs) * c.nl;
  b.base = cell0 * c.N * c.N + static_cast<int64_t>(b.zs) * c.t * c.N + static_cast<int64_t>(b.zt) * c.t;
  return b;
}

// element offset of footprint f relative to footprint 0
__device__ __forceinline__ int64_t footprint_offset(const ClusterArgs& c, int f) {
  const int du = f / (c.cs * c.nl), dv = (f / c.nl) % c.cs, l = f % c.nl;
  return ((static_cast<int64_t>(du) * c.nv + dv) * c.nl + l) * c.N * c.N;
}

// element offset of bin ab = a t + b inside the block
__device__ __forceinline__ int64_t bin_offset(const ClusterArgs& c, int ab) {
  return static_cast<int64_t>(ab / c.t) * c.N + ab % c.t;
}

// Blank image blocks (Sec. 4.2 throws complete blank ones away): one wave
// per footprint at a time sums |D| over the block's bins; the non-blank flag
// (1 or 0) goes to the first entry of the footprint's row of the Z output,
// where the ALS kernel reads it before it writes the factors.
constexpr int kMassThreads = 256;

template <typename TT>
__global__ __launch_bounds__(kMassThreads) void k_cluster_mass(ClusterArgs c) {
  const int tensor = blockIdx.x;
  const BlockPos bp = block_pos(c, tensor);
  const TT* Tb = static_cast<const TT*>(c.T) + bp.base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = kMassThreads / 64;
  const int tt = c.t * c.t, L = c.L;
  const int64_t tout = tensor * c.tmul + c.tadd;
  float* flags = c.zidx ? nullptr : c.Z + tout * L * c.R;
  int32_t* fidx = c.zidx ? c.zidx + tout * L : nullptr;
  int64_t boff[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ab = lane + 64 * q;
    boff[q] = ab < tt ? bin_offset(c, ab) : -1;
  }
  for (int f0 = wave * 4; f0 < L; f0 += nw * 4) {
    TT v[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = f0 + u;
      const int64_t fo = f < L ? footprint_offset(c, f) : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) v[u][q] = (f < L && boff[q] >= 0) ? Tb[fo + boff[q]] : TT(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      double m = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) m += fabs(static_cast<double>(v[u][q]));
      m = glint_wave_sum(m);
      if (lane == 0 && f0 + u < L) {
        if (fidx) {
          fidx[f0 + u] = m > kBlankTol ? 1 : 0;
          if (m > kBlankTol) atomicAdd(&c.counts[tout], 1);
        } else {
          flags[static_cast<int64_t>(f0 + u) * c.R] = m > kBlankTol ? 1.0f : 0.0f;
        }
      }
    }
  }
}

// lane k's value of x in every lane (k uniform)
__device__ __forceinline__ double lane_bcast(double x, int k) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffll), k);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), k);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Rank 32: Gm = (G1 o G2 + mu I)^-1 directly, by Gauss-Jordan elimination
// without pivoting (the matrix is symmetric positive definite) on wavefront
// 0 alone, lane j holding column j in registers: at step k the pivot column
// reaches every lane by readlane, so no step waits on LDS or a barrier
// (Cholesky, the inverse of its factor and their product took three passes
// of 2R workgroup barriers each; passing the column through LDS instead
// measured 8x slower).  The pivot of step k is the diagonal entry
// of the Schur complement, the quantity the Cholesky rule tests: a pivot <=
// kPivotRtol times the diagonal entry of the unfactored matrix is a
// breakdown (returns false, the same for every thread).
template <int R>
__device__ bool hadamard_inverse(const double* G1, const double* G2, double* Gm, int* flag) {
  static_assert(R <= 64, "one column per lane");
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const int j = lane < R ? lane : R - 1;     // lanes past R mirror the last column, never stored
    double a[R];
#pragma unroll
    for (int i = 0; i < R; ++i) a[i] = G1[i * R + j] * G2[i * R + j];
    double d = 0.0;     // this column's diagonal entry
#pragma unroll
    for (int i = 0; i < R; ++i) d = (i == j) ? a[i] : d;
    const double tr = glint_wave_sum(lane < R ? d : 0.0);
    const double mu = kRidgeRtol * tr / R;
    d += mu;
#pragma unroll
    for (int i = 0; i < R; ++i) a[i] = (i == j) ? d : a[i];
    int ok = 1;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const double p = lane_bcast(a[k], k);      // pivot A[k][k]
      const double dk = lane_bcast(d, k);        // its entry before elimination
      if (!(p > kPivotRtol * dk)) {
        ok = 0;
        break;
      }
      const double inv = 1.0 / p;
      const bool is_k = j == k;
      const double tk = a[k] * inv;             // new row k entry of this column
#pragma unroll
      for (int i = 0; i < R; ++i) {
        if (i == k) continue;
        const double c = lane_bcast(a[i], k);    // A[i][k] before this step
        a[i] = is_k ? -c * inv : fma(-c, tk, a[i]);
      }
      a[k] = is_k ? inv : tk;
    }
    if (ok && lane < R) {
#pragma unroll
      for (int i = 0; i < R; ++i) Gm[i * R + lane] = a[i];
    }
    if (lane == 0) *flag = ok;
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(*flag) != 0;
}

// Gm = G1 o G2 + mu I, mu = kRidgeRtol * trace(G1 o G2) / R, factored in
// place as L L^T (lower, row-major), right-looking: at step j the pivot is
// the updated diagonal entry, column j is scaled by its square root and the
// trailing lower triangle takes the rank-1 update, spread over the whole
// workgroup with a barrier after each of the two phases of a step (on one
// wavefront the update is R^2/64 dependent LDS round trips per step).  A
// pivot <= kPivotRtol times the diagonal entry of the unfactored matrix
// (kept in dg) is a breakdown: returns false (the same for every thread).
// Rank 32 takes hadamard_inverse and leaves G^-1 in Gm instead.
template <int R>
__device__ bool cholesky_hadamard(const double* G1, const double* G2, double* Gm, double* dg, double* dl) {
  if constexpr (R > 16) {
    // rank 32 keeps G^-1 itself in Gm (solve_rows applies it)
    __shared__ int s_ok;
    return hadamard_inverse<R>(G1, G2, Gm, &s_ok);
  }
  const int tid = threadIdx.x;
  for (int i = tid; i < R * R; i += blockDim.x) Gm[i] = G1[i] * G2[i];
  __syncthreads();
  if (tid < 64) {
    const int lane = tid;
    double tr = lane < R ? Gm[lane * R + lane] : 0.0;
    tr = glint_wave_sum(tr);
    const double mu = kRidgeRtol * tr / R;
    if (lane < R) {
      const double d0 = Gm[lane * R + lane] + mu;
      Gm[lane * R + lane] = d0;
      dg[lane] = d0;
    }
  }
  __syncthreads();
  int ok = 1;
  for (int j = 0; j < R; ++j) {
    const double d = Gm[j * R + j];
    // every thread reads the same values: the decision is uniform
    if (!__builtin_amdgcn_readfirstlane(static_cast<int>(d > kPivotRtol * dg[j]))) {
      ok = 0;
      break;
    }
    const double ljj = sqrt(d);
    if (tid == 0) dl[j] = ljj;
    for (int i = j + 1 + tid; i < R; i += blockDim.x) Gm[i * R + j] /= ljj;
    __syncthreads();
    for (int idx = tid; idx < R * R; idx += blockDim.x) {
      const int i = idx / R, k = idx % R;
      if (k > j && k <= i) Gm[idx] -= Gm[i * R + j] * Gm[k * R + j];
    }
    __syncthreads();
  }
  if (ok && tid < R) Gm[tid * R + tid] = dl[tid];
  __syncthreads();
  return ok != 0;
}

// A = M G^-1 for `rows` rows of stride ld, in place.
// Up to rank 16 (Lc = the Cholesky factor L of G): one row per thread,
// forward substitution L y = m then back substitution L^T x = y in
// registers.  The empty asm statements are compiler-only barriers that keep
// each step's reads of the factor at that step (hoisted, the R x R factor
// would occupy R*R registers).
// Rank 32 (Lc = G^-1 itself, from hadamard_inverse): the rows would hold 32
// FP64 registers each, and a substitution spread over lanes runs 2R
// dependent steps per row; instead every row is multiplied by G^-1 on the
// matrix cores, 16 rows per wavefront at a time.  Both give M G^-1 to
// within the conditioning of G (which the ridge bounds).
template <int R>
__device__ void apply_inverse(double* Mrows, int rows, int ld, const double* Gi) {
  static_assert(R % 16 == 0, "rank must be a multiple of 16");
  constexpr int RB = R / 16;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  for (int r0 = wave * 16; r0 < rows; r0 += nw * 16) {
    const int row = r0 + li;
    double a[R / 4];
#pragma unroll
    for (int s = 0; s < R / 4; ++s) a[s] = row < rows ? Mrows[row * ld + 4 * s + lk] : 0.0;
    f64x4 acc[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[rb] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < R / 4; ++s)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) acc[rb] = mfma64(a[s], Gi[(4 * s + lk) * R + rb * 16 + li], acc[rb]);
    // every read of these 16 rows is in registers: overwrite them
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = r0 + lk + 4 * q;
        if (i < rows) Mrows[i * ld + rb * 16 + li] = acc[rb][q];
      }
  }
}

template <int R>
__device__ void solve_rows(double* Mrows, int rows, int ld, const double* Lc) {
  if constexpr (R > 16) {
    apply_inverse<R>(Mrows, rows, ld, Lc);
    return;
  }
  for (int row = threadIdx.x; row < rows; row += blockDim.x) {
    double* m = Mrows + row * ld;
    double y[R];
#pragma unroll
    for (int k = 0; k < R; ++k) y[k] = m[k];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      asm volatile("" ::: "memory");
      double s = y[k];
#pragma unroll
      for (int i = 0; i < k; ++i) s -= Lc[k * R + i] * y[i];
      y[k] = s / Lc[k * R + k];
    }
#pragma unroll
    for (int k = R - 1; k >= 0; --k) {
      asm volatile("" ::: "memory");
      double s = y[k];
#pragma unroll
      for (int i = k + 1; i < R; ++i) s -= Lc[i * R + k] * y[i];
      y[k] = s / Lc[k * R + k];
    }
#pragma unroll
    for (int k = 0; k < R; ++k) m[k] = y[k];
  }
}

// G = F^T F for F [rows][R] (row stride ld) in LDS on the matrix cores: the
// R x R result in 16 x 16 tiles, the rows split over the waves, the waves'
// partial tiles summed through `part` (kGramPart doubles).
template <int R>
__device__ void gram_mfma(const double* F, int rows, int ld, double* G, double* part) {
  constexpr int RB = (R + 15) / 16, TILES = RB * RB, KG = kClWaves / TILES;
  static_assert(KG * TILES * 256 <= kGramPart, "Gram partials exceed their scratch");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tile = wave % TILES, kg = wave / TILES;
  if (kg < KG) {
    const int ci = (tile / RB) * 16 + li, cj = (tile % RB) * 16 + li;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    const int nsteps = (rows + 3) / 4;
    for (int s = kg; s < nsteps; s += KG) {
      const int row = s * 4 + lk;
      const double a = (row < rows && ci < R) ? F[row * ld + ci] : 0.0;
      const double b = (row < rows && cj < R) ? F[row * ld + cj] : 0.0;
      acc = mfma64(a, b, acc);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) part[(kg * TILES + tile) * 256 + (lk + 4 * q) * 16 + li] = acc[q];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) {
    const int r = idx / R, q = idx % R;
    const int tl = (r / 16) * RB + q / 16;
    double s = 0.0;
    for (int g = 0; g < KG; ++g) s += part[(g * TILES + tl) * 256 + (r % 16) * 16 + q % 16];
    G[idx] = s;
  }
  __syncthreads();
}

// Columns of F to unit length (zero columns stay zero), lam[r] = the norms,
// and G (= F^T F on entry) to the Gram of the normalised F.
template <int R>
__device__ void normalize_by_gram(double* F, int rows, int ld, double* G, double* lam) {
  if (threadIdx.x < R) lam[threadIdx.x] = sqrt(G[threadIdx.x * R + threadIdx.x]);
  __syncthreads();
  for (int idx = threadIdx.x; idx < rows * R; idx += blockDim.x) {
    const int row = idx / R, r = idx % R;
    const double n = lam[r];
    if (n > 0.0) F[row * ld + r] /= n;
  }
  for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) {
    const double nr = lam[idx / R], nq = lam[idx % R];
    if (nr > 0.0 && nq > 0.0) G[idx] = G[idx] / nr / nq;
  }
  __syncthreads();
}

// CP-ALS of one block tensor by the whole workgroup (every sweep).  Not
// inlined: its early exits then stay inside the call, and the persistent
// loop around it is a plain scalar loop.
template <typename TT, int R, bool ZG>
__device__ __noinline__ void als_one(const ClusterArgs& c, int tensor) {
  constexpr int RB = (R + 15) / 16;
  constexpr int ABC = stage_ab<TT>(), SS = stage_stride<TT>();
  constexpr int PER = kFR * ABC / kClThreads;     // staged elements per thread per chunk
  static_assert(kClThreads % ABC == 0, "stage rows must map to fixed lanes");
  extern __shared__ __align__(16) double cl_lds[];
  const int t = c.t, L = c.L, tt = t * t, ZS = R + 1;
  const ClusterLds o = cluster_lds(t, L, R, stage_doubles<TT>(), ZG);
  double* X = cl_lds + o.x;
  double* Y = cl_lds + o.y;
  double* Mt = cl_lds + o.mt;
  double* Z = ZG ? c.zws + static_cast<int64_t>(blockIdx.x) * c.zws_stride : cl_lds + o.z;
  double* P = cl_lds + o.p;
  double* GX = cl_lds + o.gx;
  double* GY = cl_lds + o.gy;
  double* GZ = cl_lds + o.gz;
  double* Gm = cl_lds + o.gm;
  double* lam = cl_lds + o.lam;
  double* dg = cl_lds + o.dg;
  double* dl = cl_lds + o.dl;
  int64_t* foff = reinterpret_cast<int64_t*>(cl_lds + o.foff);
  TT* stage = reinterpret_cast<TT*>(cl_lds + o.stage);
  double* part = cl_lds + o.stage;

  int* keep = reinterpret_cast<int*>(cl_lds + o.keep);
  int* rowof = reinterpret_cast<int*>(cl_lds + o.rowof);
  __shared__ int wcnt[kClWaves];

  const int64_t tout = tensor * c.tmul + c.tadd;
  float* outX = c.X + tout * t * R;
  float* outY = c.Y + tout * t * R;
  float* outZ = c.zidx ? nullptr : c.Z + tout * L * R;      // dense layout
  const int32_t* zrow = c.zidx ? c.zidx + tout * L : nullptr;  // compact layout
  const BlockPos bp = block_pos(c, tensor);
  const TT* Tb = static_cast<const TT*>(c.T) + bp.base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;

  // blank image blocks are thrown away: the flags k_cluster_mass left in the
  // Z rows (or the compact layout's row index), then the non-blank
  // footprints are stacked in order
  for (int f = threadIdx.x; f < L; f += blockDim.x)
    rowof[f] = zrow ? (zrow[f] >= 0 ? 1 : 0) : (outZ[static_cast<int64_t>(f) * R] != 0.0f ? 1 : 0);
  __syncthreads();
  int Lc = 0;
  for (int base = 0; base < L; base += kClThreads) {
    const int f = base + static_cast<int>(threadIdx.x);
    const bool nb = f < L && rowof[f] != 0;
    const unsigned long long bal = __ballot(nb);
    if (lane == 0) wcnt[wave] = __popcll(bal);
    __syncthreads();
    int off = Lc, tot = 0;
    for (int w = 0; w < kClWaves; ++w) {
      if (w < wave) off += wcnt[w];
      tot += wcnt[w];
    }
    if (f < L) {
      const int j = off + __popcll(bal & ((1ull << lane) - 1ull));
      if (nb) keep[j] = f;
      rowof[f] = nb ? j : -1;
    }
    Lc += __builtin_amdgcn_readfirstlane(tot);     // uniform: it decides branches around barriers
    __syncthreads();
  }
  if (Lc == 0) {
    for (int i = threadIdx.x; i < t * R; i += blockDim.x) {
      outX[i] = 0.0f;
      outY[i] = 0.0f;
    }
    if (outZ)
      for (int i = threadIdx.x; i < L * R; i += blockDim.x) outZ[i] = 0.0f;
    if (threadIdx.x == 0) {
      c.blank[tout] = 1;
      atomicAdd(&c.info[1], 1);
    }
    return;
  }

  // offsets of the stacked footprints, initial factors (SplitMix64 counters;
  // a Z row is numbered by its footprint), lambda = 1
  for (int j = threadIdx.x; j < Lc; j += blockDim.x) foff[j] = footprint_offset(c, keep[j]);
  const uint64_t rows_max = t > L ? t : L;
  for (int i = threadIdx.x; i < t * R; i += blockDim.x) {
    const uint64_t row = i / R, r = i % R;
    X[i] = glint_sm64_uniform(c.seed, ((static_cast<uint64_t>(tout) * 3 + 0) * rows_max + row) * R + r);
    Y[i] = glint_sm64_uniform(c.seed, ((static_cast<uint64_t>(tout) * 3 + 1) * rows_max + row) * R + r);
  }
  for (int i = threadIdx.x; i < Lc * R; i += blockDim.x) {
    const int j = i / R, r = i % R;
    const uint64_t row = static_cast<uint64_t>(keep[j]);
    Z[j * ZS + r] = glint_sm64_uniform(c.seed, ((static_cast<uint64_t>(tout) * 3 + 2) * rows_max + row) * R + r);
  }
  if (threadIdx.x < R) lam[threadIdx.x] = 1.0;
  __syncthreads();
  gram_mfma<R>(X, t, R, GX, part);
  gram_mfma<R>(Y, t, R, GY, part);
  gram_mfma<R>(Z, Lc, ZS, GZ, part);

  // pass A: this wave's bin blocks (16 bins each) are `wave` and `wave + 8`
  const int nabb = (tt + 15) / 16;
  int64_t aoff[2];
  bool aok[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int ab = (wave + kClWaves * b) * 16 + li;
    aok[b] = ab < tt;
    aoff[b] = aok[b] ? bin_offset(c, ab) : 0;
  }
  const bool own0 = wave < nabb, own1 = wave + kClWaves < nabb;
  constexpr int kUK = pass_a_batch<TT>();
  const int nsteps_a = (Lc + 3) / 4;
  const int nbatch_a = (nsteps_a + kUK - 1) / kUK;
  // pass B: the staged element e of this thread is bin (chunk start + sab),
  // footprint (range start + sf0 + e * (kClThreads / ABC))
  const int sab = threadIdx.x % ABC, sf0 = threadIdx.x / ABC;
  const int nabc = (tt + ABC - 1) / ABC;
  const int nchunk_b = ((Lc + kFR - 1) / kFR) * nabc;
  int fails = 0;

  for (int it = 0; it < c.iters; ++it) {
    // ---- pass A: P[ab][r] = sum_f D[ab][f] Z[f][r] ----
    {
      f64x4 acc[2][RB];
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[b][rb] = f64x4{0.0, 0.0, 0.0, 0.0};
      TT cur[kUK][2], nxt[kUK][2];
      // with Z in global memory its rows are fetched with the batch's D
      constexpr int ZB = ZG ? kUK : 1;
      double zc[ZB][RB], zn[ZB][RB];
      auto load = [&](int batch, TT (&v)[kUK][2], double (&zv)[ZB][RB]) {
#pragma unroll
        for (int s = 0; s < kUK; ++s) {
          const int f = (batch * kUK + s) * 4 + lk;
          const bool fok = f < Lc;
          const int64_t fo = fok ? foff[f] : 0;
#pragma unroll
          for (int b = 0; b < 2; ++b) v[s][b] = (fok && aok[b]) ? Tb[fo + aoff[b]] : TT(0);
          if constexpr (ZG) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) zv[s][rb] = (fok && rb * 16 + li < R) ? Z[f * ZS + rb * 16 + li] : 0.0;
          }
        }
      };
      if (own0) load(0, cur, zc);
      for (int bt = 0; bt < nbatch_a; ++bt) {
        if (own0 && bt + 1 < nbatch_a) load(bt + 1, nxt, zn);
        if (own0) {
#pragma unroll
          for (int s = 0; s < kUK; ++s) {
            const int f = (bt * kUK + s) * 4 + lk;
            double bz[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
              if constexpr (ZG) bz[rb] = zc[s][rb];
              else bz[rb] = (f < Lc && rb * 16 + li < R) ? Z[f * ZS + rb * 16 + li] : 0.0;
            }
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[0][rb] = mfma64(static_cast<double>(cur[s][0]), bz[rb], acc[0][rb]);
            if (own1) {
#pragma unroll
              for (int rb = 0; rb < RB; ++rb) acc[1][rb] = mfma64(static_cast<double>(cur[s][1]), bz[rb], acc[1][rb]);
            }
          }
#pragma unroll
          for (int s = 0; s < kUK; ++s) {
            cur[s][0] = nxt[s][0];
            cur[s][1] = nxt[s][1];
          }
          if constexpr (ZG) {
#pragma unroll
            for (int s = 0; s < kUK; ++s)
#pragma unroll
              for (int rb = 0; rb < RB; ++rb) zc[s][rb] = zn[s][rb];
          }
        }
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (b == 0 ? !own0 : !own1) continue;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int ab = (wave + kClWaves * b) * 16 + lk + 4 * q, r = rb * 16 + li;
            if (ab < tt && r < R) P[ab * R + r] = acc[b][rb][q];
          }
      }
    }
    __syncthreads();
    // ---- mode X: M[a][r] = sum_b P[ab][r] Y[b][r] ----
    for (int idx = threadIdx.x; idx < t * R; idx += blockDim.x) {
      const int a = idx / R, r = idx % R;
      double s = 0.0;
      for (int b = 0; b < t; ++b) s += P[(a * t + b) * R + r] * Y[b * R + r];
      Mt[idx] = s;
    }
    __syncthreads();
    if (cholesky_hadamard<R>(GY, GZ, Gm, dg, dl)) {
      solve_rows<R>(Mt, t, R, Gm);
      __syncthreads();
      for (int i = threadIdx.x; i < t * R; i += blockDim.x) X[i] = Mt[i];
      __syncthreads();
      gram_mfma<R>(X, t, R, GX, part);
      normalize_by_gram<R>(X, t, R, GX, lam);
    } else {
      ++fails;
    }
    // ---- mode Y: M[b][r] = sum_a P[ab][r] X[a][r] ----
    for (int idx = threadIdx.x; idx < t * R; idx += blockDim.x) {
      const int b = idx / R, r = idx % R;
      double s = 0.0;
      for (int a = 0; a < t; ++a) s += P[(a * t + b) * R + r] * X[a * R + r];
      Mt[idx] = s;
    }
    __syncthreads();
    if (cholesky_hadamard<R>(GX, GZ, Gm, dg, dl)) {
      solve_rows<R>(Mt, t, R, Gm);
      __syncthreads();
      for (int i = threadIdx.x; i < t * R; i += blockDim.x) Y[i] = Mt[i];
      __syncthreads();
      gram_mfma<R>(Y, t, R, GY, part);
      normalize_by_gram<R>(Y, t, R, GY, lam);
    } else {
      ++fails;
    }
    // ---- mode Z (factored first: Z is overwritten in place only when it succeeds) ----
    if (cholesky_hadamard<R>(GX, GY, Gm, dg, dl)) {
      for (int idx = threadIdx.x; idx < tt * R; idx += blockDim.x) {
        const int ab = idx / R, r = idx % R;
        P[idx] = X[(ab / t) * R + r] * Y[(ab % t) * R + r];      // Khatri-Rao of X and Y
      }
      // pass B: Z[f][r] = sum_ab D[ab][f] P[ab][r], footprint ranges of kFR,
      // bin chunks of ABC staged through LDS; wave w owns footprints 16w..16w+15
      auto sload = [&](int chunk, TT (&reg)[PER]) {
        const int fr = (chunk / nabc) * kFR, a0 = (chunk % nabc) * ABC;
        const int ab = a0 + sab;
        const int64_t bo = ab < tt ? bin_offset(c, ab) : 0;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
          const int f = fr + sf0 + e * (kClThreads / ABC);
          reg[e] = (f < Lc && ab < tt) ? Tb[foff[f] + bo] : TT(0);
        }
      };
      f64x4 accz[RB];
      // one chunk: stage it, refill its registers with the chunk two ahead,
      // then run this wave's 16 footprints through the matrix cores
      auto chunk_step = [&](int ch, TT (&reg)[PER]) {
        const int fr = (ch / nabc) * kFR, a0 = (ch % nabc) * ABC;
#pragma unroll
        for (int e = 0; e < PER; ++e) stage[(sf0 + e * (kClThreads / ABC)) * SS + sab] = reg[e];
        __syncthreads();
        if (ch + 2 < nchunk_b) sload(ch + 2, reg);
        if (a0 == 0) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) accz[rb] = f64x4{0.0, 0.0, 0.0, 0.0};
        }
        const int f0 = fr + wave * 16;
        if (f0 < Lc) {
#pragma unroll 4
          for (int s = 0; s < ABC / 4; ++s) {
            const int ab = a0 + s * 4 + lk;
            const double a = static_cast<double>(stage[(wave * 16 + li) * SS + s * 4 + lk]);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
              const double b = (ab < tt && rb * 16 + li < R) ? P[ab * R + rb * 16 + li] : 0.0;
              accz[rb] = mfma64(a, b, accz[rb]);
            }
          }
          if (a0 + ABC >= tt) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int f = f0 + lk + 4 * q, r = rb * 16 + li;
                if (f < Lc && r < R) Z[f * ZS + r] = accz[rb][q];
              }
          }
        }
        __syncthreads();
      };
      TT ra[PER], rb2[PER];
      sload(0, ra);
      if (nchunk_b > 1) sload(1, rb2);
      for (int ch = 0; ch < nchunk_b; ch += 2) {
        chunk_step(ch, ra);
        if (ch + 1 < nchunk_b) chunk_step(ch + 1, rb2);
      }
      solve_rows<R>(Z, Lc, ZS, Gm);
      __syncthreads();
      gram_mfma<R>(Z, Lc, ZS, GZ, part);
      normalize_by_gram<R>(Z, Lc, ZS, GZ, lam);
    } else {
      ++fails;
    }
  }
  // outputs: X, Y, Z * lambda (FP32)
  for (int i = threadIdx.x; i < t * R; i += blockDim.x) {
    outX[i] = static_cast<float>(X[i]);
    outY[i] = static_cast<float>(Y[i]);
  }
  if (outZ) {
    for (int i = threadIdx.x; i < L * R; i += blockDim.x) {
      const int f = i / R, r = i % R, j = rowof[f];
      outZ[i] = j >= 0 ? static_cast<float>(Z[j * ZS + r] * lam[r]) : 0.0f;
    }
  } else {
    for (int i = threadIdx.x; i < Lc * R; i += blockDim.x) {
      const int j = i / R, r = i % R;
      c.Z[static_cast<int64_t>(zrow[keep[j]]) * R + r] = static_cast<float>(Z[j * ZS + r] * lam[r]);
    }
  }
  if (threadIdx.x == 0) {
    c.blank[tout] = 0;
    atomicAdd(&c.info[3], Lc);
  }
  if (threadIdx.x == 0 && fails) atomicAdd(&c.info[0], fails);
}

// Persistent workgroups (as many as fit on the chip at once) take block
// tensors from a counter (info[2]) until all are done: blank blocks cost only
// their zero outputs, and a fixed index-to-tensor mapping would let the
// workgroup dispatcher's round-robin over XCDs and shader engines line up
// with the angular positions of the non-blank blocks.
template <typename TT, int R, bool ZG>
__global__ __launch_bounds__(kClThreads) void k_cluster_als(ClusterArgs c) {
  __shared__ int s_next;
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(&c.info[2], 1);
    __syncthreads();
    // the same value in every lane: made wave-uniform so that the loop exit
    // and everything below stay scalar branches (a per-lane exit would put
    // the claiming lane under an exec mask on the next trip)
    const int tensor = __builtin_amdgcn_readfirstlane(s_next);
    __syncthreads();
    if (tensor >= c.ntensor) break;
    als_one<TT, R, ZG>(c, tensor);
  }
}

__global__ void k_cluster_info_init(int* info) {
  if (threadIdx.x < 4) info[threadIdx.x] = 0;
}

__global__ void k_cluster_claim_reset(int* info) {
  if (threadIdx.x == 0) info[2] = 0;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Exclusive prefix sum of the per-tensor counts into the compact rows'
// bases: base[i] = sum_{j<i} counts[j], base[n] = the total.  Three steps
// over chunks of kScanChunk counts: chunk sums, one workgroup scanning the
// chunk sums in order (a running carry), and the scan inside each chunk.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanChunk = kScanThreads * kScanPer;

// exclusive scan of v over the workgroup (kScanThreads threads); *total = the sum
__device__ int64_t block_exclusive_scan(int64_t v, int64_t* total) {
  __shared__ int64_t wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t o = __shfl_up(inc, d);
    if (lane >= d) inc += o;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  int64_t before = 0, all = 0;
  for (int w = 0; w < kScanThreads / 64; ++w) {
    if (w < wave) before += wsum[w];
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_chunks(const int32_t* __restrict__ counts, int64_t n,
                                                              int64_t* __restrict__ csum) {
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kScanChunk + threadIdx.x * kScanPer;
  int64_t v = 0;
#pragma unroll
  for (int e = 0; e < kScanPer; ++e)
    if (i0 + e < n) v += counts[i0 + e];
  int64_t total;
  block_exclusive_scan(v, &total);
  if (threadIdx.x == 0) csum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(int64_t* __restrict__ csum, int64_t nchunk,
                                                           int64_t* __restrict__ base, int64_t n, int* info) {
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nchunk; c0 += kScanThreads) {
    const int64_t c = c0 + threadIdx.x;
    const int64_t v = c < nchunk ? csum[c] : 0;
    int64_t total;
    const int64_t ex = block_exclusive_scan(v, &total);
    if (c < nchunk) csum[c] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) {
    base[n] = carry;
    info[3] = carry < 0x7fffffff ? static_cast<int>(carry) : 0x7fffffff;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t* __restrict__ counts, int64_t n,
                                                             const int64_t* __restrict__ csum,
                                                             int64_t* __restrict__ base) {
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kScanChunk + threadIdx.x * kScanPer;
  int64_t v = 0;
#pragma unroll
  for (int e = 0; e < kScanPer; ++e)
    if (i0 + e < n) v += counts[i0 + e];
  int64_t total;
  int64_t run = csum[blockIdx.x] + block_exclusive_scan(v, &total);
#pragma unroll
  for (int e = 0; e < kScanPer; ++e)
    if (i0 + e < n) {
      base[i0 + e] = run;
      run += counts[i0 + e];
    }
}

// The compact rows: one wavefront per tensor turns the mass pass's 0/1
// flags in zidx[tensor][f] into base[tensor] + (the footprint's place among
// the tensor's non-blank footprints), or -1; a tensor without any counts
// as blank (info[1]).
__global__ __launch_bounds__(256) void k_cluster_rows(int32_t* __restrict__ zidx, const int64_t* __restrict__ base,
                                                      int64_t ntensor, int L, int* info) {
  const int lane = threadIdx.x & 63;
  const int64_t tensor = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  if (tensor >= ntensor) return;
  int32_t* z = zidx + tensor * L;
  const int64_t b = base[tensor];
  int run = 0;
  for (int f0 = 0; f0 < L; f0 += 64) {
    const int f = f0 + lane;
    const bool nb = f < L && z[f] != 0;
    const unsigned long long bal = __ballot(nb);
    if (f < L) z[f] = nb ? static_cast<int32_t>(b + run + __popcll(bal & ((1ull << lane) - 1ull))) : -1;
    run += __popcll(bal);
  }
  if (lane == 0 && run == 0) atomicAdd(&info[1], 1);
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
  const void* CX;    // [ntensor][t+1][R], FP32 or BF16
  const void* CY;
  const void* Z;     // [ntensor][L][R], or [rows][R] with zidx
  const int32_t* zidx;   // compact layout: [ntensor][L] row of Z or -1 (blank)
  int t, cs, nu, nv, nl, N, ncv, nb, L;
  int64_t nq;
  const int32_t* q;
  float* out;
};

// A resolved record of the clustered query: the region's first tensor, the
// footprint, the clamped box, and the Z rows of the first kClPre blocks the
// box overlaps (zs-major), looked up by the lane that resolves the record so
// that the row-index loads of a wave's 64 records are in flight together
// (measured at 2048^2, rank 32, compact Z: 6.3 G queries/s with the row
// loaded inside the block loop, 8.5 / 9.4 / 8.2 with 1 / 2 / 4 blocks
// resolved ahead; more blocks cost occupancy).
constexpr int kClPre = 2;

struct alignas(16) ClRec {
  int tensor0;   // tensor index of block (0, 0) of the region
  int f;
  int slo, shi, tlo, thi;
  int nblk;      // blocks the box overlaps (0: empty box)
  int pad;
  int64_t rows[kClPre];   // Z row of each of the first kClPre blocks, -1 for a blank one
};

constexpr int kClQueryThreads = 256;

__device__ __forceinline__ int64_t cl_row(const ClQueryArgs& a, int64_t tensor, int f) {
  const int64_t zr = tensor * a.L + f;
  return a.zidx ? static_cast<int64_t>(a.zidx[zr]) : zr;
}

// A lane's RPL consecutive values of a table row: FP32 kept as loaded, BF16
// kept as the loaded words (one 16-byte load for eight ranks, 8 bytes for
// four; rows aligned to that) and decoded exactly to FP32 where used.
template <typename ET, int RPL>
struct ClRow {
  float v[RPL];
  __device__ __forceinline__ void load(const float* p) {
#pragma unroll
    for (int e = 0; e < RPL; ++e) v[e] = p[e];
  }
  __device__ __forceinline__ float operator[](int e) const { return v[e]; }
};

template <int RPL>
struct ClRow<uint16_t, RPL> {
  static_assert(RPL == 4 || RPL == 8, "BF16 rows: 4 or 8 ranks a lane");
  uint32_t w[RPL / 2];
  __device__ __forceinline__ void load(const uint16_t* p) {
    if constexpr (RPL == 8) {
      const uint4 x = *reinterpret_cast<const uint4*>(p);
      w[0] = x.x; w[1] = x.y; w[2] = x.z; w[3] = x.w;
    } else {
      const uint2 x = *reinterpret_cast<const uint2*>(p);
      w[0] = x.x; w[1] = x.y;
    }
  }
  __device__ __forceinline__ float operator[](int e) const {
    return (e & 1) ? __uint_as_float(w[e >> 1] & 0xffff0000u) : __uint_as_float(w[e >> 1] << 16);
  }
};

// Ranks a lane of the clustered query: 16 bytes of a row (FP32: 4, BF16: 8,
// BF16 rank 4: 4).
template <typename ET, int R>
constexpr int cl_rpl() {
  return sizeof(ET) == 2 && R >= 8 ? 8 : 4;
}

// lane group of LPQ = R / RPL lanes per query, RPL ranks per lane.
// Phase 1: lane i resolves record base + i (and its first blocks' Z rows);
// phase 2: group g serves records g*LPQ .. g*LPQ + LPQ - 1, loading the rows
// of the first kClPre blocks of a box together before any arithmetic.  The
// blocks' terms are added in zs-major order, ranks in order within a block.
template <typename ET, int R>
__global__ __launch_bounds__(kClQueryThreads) void k_query_clustered(ClQueryArgs a) {
  constexpr int RPL = cl_rpl<ET, R>();
  static_assert(R % RPL == 0, "rank a multiple of the ranks a lane");
  const ET* __restrict__ CXg = static_cast<const ET*>(a.CX);
  const ET* __restrict__ CYg = static_cast<const ET*>(a.CY);
  const ET* __restrict__ Zg = static_cast<const ET*>(a.Z);
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
      // records and results stream through once (non-temporal), the table
      // rows stay in the caches for the footprint's other boxes
      int f[7];
#pragma unroll
      for (int e = 0; e < 7; ++e) f[e] = __builtin_nontemporal_load(rec + e);
      const int u = glint_wrap(f[0], a.nu), v = glint_wrap(f[1], a.nv);
      const int l = glint_clampi(f[2], 0, a.nl - 1);
      ClRec cr;
      cr.tensor0 = ((u / a.cs) * a.ncv + v / a.cs) * a.nb * a.nb;
      cr.f = ((u % a.cs) * a.cs + v % a.cs) * a.nl + l;
      cr.slo = glint_clampi(f[3], 0, a.N);
      cr.shi = glint_clampi(f[4], 0, a.N);
      cr.tlo = glint_clampi(f[5], 0, a.N);
      cr.thi = glint_clampi(f[6], 0, a.N);
      cr.pad = 0;
      cr.nblk = 0;
      const bool nonempty = cr.slo < cr.shi && cr.tlo < cr.thi;
      const int zs0 = cr.slo / t, zt0 = cr.tlo / t;
      const int nzt = nonempty ? (cr.thi - 1) / t - zt0 + 1 : 0;
      if (nonempty) cr.nblk = ((cr.shi - 1) / t - zs0 + 1) * nzt;
#pragma unroll
      for (int b = 0; b < kClPre; ++b) {
        cr.rows[b] = -1;
        if (b < cr.nblk) cr.rows[b] = cl_row(a, cr.tensor0 + (zs0 + b / nzt) * a.nb + zt0 + b % nzt, cr.f);
      }
      wr[lane] = cr;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    float res = 0.0f;
    for (int jj = 0; jj < LPQ; ++jj) {
      const ClRec cr = wr[g * LPQ + jj];
      float acc = 0.0f;
      if (cr.nblk > 0) {
        const int zs0 = cr.slo / t, zt0 = cr.tlo / t;
        const int nzt = (cr.thi - 1) / t - zt0 + 1;
        // the first kClPre blocks: every row loaded before the arithmetic
        ClRow<ET, RPL> zz[kClPre], xh[kClPre], xl[kClPre], yh[kClPre], yl[kClPre];
#pragma unroll
        for (int b = 0; b < kClPre; ++b) {
          if (b < cr.nblk && cr.rows[b] >= 0) {
            const int zs = zs0 + b / nzt, zt = zt0 + b % nzt;
            const int a0 = max(cr.slo, zs * t) - zs * t, a1 = min(cr.shi, (zs + 1) * t) - zs * t;
            const int b0 = max(cr.tlo, zt * t) - zt * t, b1 = min(cr.thi, (zt + 1) * t) - zt * t;
            const int64_t tensor = cr.tensor0 + zs * a.nb + zt;
            const ET* cx = CXg + tensor * (t + 1) * R + r0;
            const ET* cy = CYg + tensor * (t + 1) * R + r0;
            zz[b].load(Zg + cr.rows[b] * R + r0);
            xh[b].load(cx + a1 * R);
            xl[b].load(cx + a0 * R);
            yh[b].load(cy + b1 * R);
            yl[b].load(cy + b0 * R);
          }
        }
#pragma unroll
        for (int b = 0; b < kClPre; ++b) {
          if (b < cr.nblk && cr.rows[b] >= 0) {
#pragma unroll
            for (int e = 0; e < RPL; ++e) acc += zz[b][e] * (xh[b][e] - xl[b][e]) * (yh[b][e] - yl[b][e]);
          }
        }
        // boxes over more blocks: the rest one by one
        for (int b = kClPre; b < cr.nblk; ++b) {
          const int zs = zs0 + b / nzt, zt = zt0 + b % nzt;
          const int64_t tensor = cr.tensor0 + zs * a.nb + zt;
          const int64_t zr = cl_row(a, tensor, cr.f);
          if (zr < 0) continue;     // blank image block: no terms
          const int a0 = max(cr.slo, zs * t) - zs * t, a1 = min(cr.shi, (zs + 1) * t) - zs * t;
          const int b0 = max(cr.tlo, zt * t) - zt * t, b1 = min(cr.thi, (zt + 1) * t) - zt * t;
          const ET* cx = CXg + tensor * (t + 1) * R + r0;
          const ET* cy = CYg + tensor * (t + 1) * R + r0;
          ClRow<ET, RPL> z, xh, xl, yh, yl;
          z.load(Zg + zr * R + r0);
          xh.load(cx + a1 * R);
          xl.load(cx + a0 * R);
          yh.load(cy + b1 * R);
          yl.load(cy + b0 * R);
#pragma unroll
          for (int e = 0; e < RPL; ++e) acc += z[e] * (xh[e] - xl[e]) * (yh[e] - yl[e]);
        }
      }
      acc = glint_group_sum<LPQ>(acc);
      res = (j == jj) ? acc : res;
    }
    __builtin_amdgcn_wave_barrier();
    const int64_t qo = base + g * LPQ + j;
    if (qo < a.nq) __builtin_nontemporal_store(res, a.out + qo);
  }
}

// ---------------------------------------------------------------------------
// hierarchical importance sampling on the clustered tables (Sec. 5.2)
// ---------------------------------------------------------------------------

struct ClSampleArgs {
  const float* CX;
  const float* CY;
  const float* Z;
  const int32_t* zidx;
  int t, cs, nu, nv, nl, N, ncv, nb, L, levels;
  int64_t n;
  const int32_t* uvl;
  const float* rnd;
  float* h;
  float* pdf;
  int32_t* bins;
};

constexpr int kClSampleThreads = 256;

// block-local range query of tensor `tensor` (footprint f) over [a0, a1) x [b0, b1)
template <int R>
__device__ __forceinline__ float cl_box(const ClSampleArgs& a, int64_t tensor, int f, int a0, int a1, int b0,
                                        int b1) {
  int64_t zr = tensor * a.L + f;
  if (a.zidx) {
    zr = a.zidx[zr];
    if (zr < 0) return 0.0f;
  }
  const float* z = a.Z + zr * R;
  const float* cx = a.CX + tensor * (a.t + 1) * R;
  const float* cy = a.CY + tensor * (a.t + 1) * R;
  float m = 0.0f;
#pragma unroll
  for (int r = 0; r < R; ++r) m += z[r] * (cx[a1 * R + r] - cx[a0 * R + r]) * (cy[b1 * R + r] - cy[b0 * R + r]);
  return m;
}

// One sample per thread: the block by its mass (running-sum rule over the
// blocks in zs-major order, negative masses as zero), then log2(t) levels of
// four quads inside it, then a uniform position in the bin.
template <int R>
__global__ __launch_bounds__(kClSampleThreads) void k_sample_clustered(ClSampleArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int u = glint_wrap(a.uvl[3 * i], a.nu), v = glint_wrap(a.uvl[3 * i + 1], a.nv);
  const int l = glint_clampi(a.uvl[3 * i + 2], 0, a.nl - 1);
  const int64_t tensor0 = (static_cast<int64_t>(u / a.cs) * a.ncv + v / a.cs) * a.nb * a.nb;
  const int f = ((u % a.cs) * a.cs + v % a.cs) * a.nl + l;
  const float* rn = a.rnd + i * (a.levels + 3);
  const int nblk = a.nb * a.nb, t = a.t;
  // up to kCachedBlocks block masses stay in registers for the search
  constexpr int kCachedBlocks = 16;
  const bool cached = nblk <= kCachedBlocks;
  float bm[kCachedBlocks];
  float total = 0.0f;
  if (cached) {
#pragma unroll
    for (int b = 0; b < kCachedBlocks; ++b) {
      bm[b] = b < nblk ? fmaxf(cl_box<R>(a, tensor0 + b, f, 0, t, 0, t), 0.0f) : 0.0f;
      total += bm[b];
    }
  } else {
    for (int b = 0; b < nblk; ++b) total += fmaxf(cl_box<R>(a, tensor0 + b, f, 0, t, 0, t), 0.0f);
  }
  a.h[2 * i] = 0.0f;
  a.h[2 * i + 1] = 0.0f;
  a.pdf[i] = 0.0f;
  a.bins[2 * i] = -1;
  a.bins[2 * i + 1] = -1;
  if (!(total > 0.0f)) return;
  const float target = rn[0] * total;
  float run = 0.0f, pm = 0.0f, lastm = 0.0f;
  int pick = -1, lastpos = 0;
  if (cached) {
#pragma unroll
    for (int b = 0; b < kCachedBlocks; ++b) {
      if (b < nblk && pick < 0) {
        const float m = bm[b];
        if (m > 0.0f) {
          lastpos = b;
          lastm = m;
        }
        run += m;
        if (target < run) {
          pick = b;
          pm = m;
        }
      }
    }
  } else {
    for (int b = 0; b < nblk; ++b) {
      const float m = fmaxf(cl_box<R>(a, tensor0 + b, f, 0, t, 0, t), 0.0f);
      if (m > 0.0f) {
        lastpos = b;
        lastm = m;
      }
      run += m;
      if (target < run) {
        pick = b;
        pm = m;
        break;
      }
    }
  }
  if (pick < 0) {
    pick = lastpos;
    pm = lastm;
  }
  float prob = pm / total;
  const int64_t tensor = tensor0 + pick;
  int s0 = 0, s1 = t, t0 = 0, t1 = t;
  for (int k = 0; k < a.levels; ++k) {
    const int sm = (s0 + s1) >> 1, tm = (t0 + t1) >> 1;
    float m[4];
    m[0] = fmaxf(cl_box<R>(a, tensor, f, s0, sm, t0, tm), 0.0f);
    m[1] = fmaxf(cl_box<R>(a, tensor, f, s0, sm, tm, t1), 0.0f);
    m[2] = fmaxf(cl_box<R>(a, tensor, f, sm, s1, t0, tm), 0.0f);
    m[3] = fmaxf(cl_box<R>(a, tensor, f, sm, s1, tm, t1), 0.0f);
    const float qt = ((m[0] + m[1]) + m[2]) + m[3];
    if (!(qt > 0.0f)) return;
    const float tq = rn[1 + k] * qt;
    int q = 3;
    float rq = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      rq += m[j];
      if (tq < rq) {
        q = j;
        break;
      }
    }
    while (m[q] <= 0.0f) --q;
    prob *= m[q] / qt;
    if (q >= 2) s0 = sm; else s1 = sm;
    if (q & 1) t0 = tm; else t1 = tm;
  }
  const int zs = pick / a.nb, zt = pick % a.nb;
  const int bs = zs * t + s0, bt = zt * t + t0;
  const float w = 2.0f / static_cast<float>(a.N);
  a.bins[2 * i] = bs;
  a.bins[2 * i + 1] = bt;
  a.h[2 * i] = -1.0f + (static_cast<float>(bs) + rn[1 + a.levels]) * w;
  a.h[2 * i + 1] = -1.0f + (static_cast<float>(bt) + rn[2 + a.levels]) * w;
  a.pdf[i] = prob / (w * w);
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
  GLINT_SUPPORT(s->ntensor < (int64_t{1} << 30), "too many region-and-block tensors");
  return GLINT_OK;
}

template <typename TT, int R>
size_t cluster_als_lds(int t, int L, bool z_global) {
  return sizeof(double) * static_cast<size_t>(cluster_lds(t, L, R, stage_doubles<TT>(), z_global).total_doubles);
}

// Z factor slots in global memory: as many as ALS workgroups can run at once
// (the kernel's LDS use allows at most this many per CU when Z is global)
constexpr int kZSlotsPerCu = 2;

// The mass pass (when asked) and the persistent ALS kernel.  Z stays in LDS
// when it fits; otherwise it goes to the zslots slots of c.zws, or the call
// is refused when there are none.
template <typename TT, int R>
glint_status launch_cluster_als(const ClusterArgs& c0, int64_t ntensor, bool run_mass, int64_t zslots,
                                hipStream_t stream) {
  ClusterArgs c = c0;
  const size_t lds_in = cluster_als_lds<TT, R>(c.t, c.L, false);
  const bool zg = static_cast<int64_t>(lds_in) + 64 > g_cl_lds;   // + the kernel's static slots
  const size_t lds = zg ? cluster_als_lds<TT, R>(c.t, c.L, true) : lds_in;
  if (static_cast<int64_t>(lds) + 64 > g_cl_lds)
    return glint_fail(GLINT_E_UNSUPPORTED, "clustered ALS needs %zu bytes of LDS (device max %d)", lds, g_cl_lds);
  if (zg && (c.zws == nullptr || zslots < 1))
    return glint_fail(GLINT_E_UNSUPPORTED,
                      "the Z factors of %d footprints at rank %d need %zu bytes of LDS (device max %d); "
                      "glint_cp_als_clustered_map keeps them in its workspace instead", c.L, R, lds_in, g_cl_lds);
  if (run_mass) {
    hipLaunchKernelGGL((k_cluster_mass<TT>), dim3(static_cast<unsigned>(ntensor)), dim3(kMassThreads), 0, stream, c);
    GLINT_LAUNCHED("k_cluster_mass");
  }
  const void* kfn = zg ? reinterpret_cast<const void*>(k_cluster_als<TT, R, true>)
                       : reinterpret_cast<const void*>(k_cluster_als<TT, R, false>);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, kClThreads, lds) != hipSuccess || per_cu < 1)
    return glint_fail(GLINT_E_HIP, "occupancy query for k_cluster_als failed");
  int64_t grid = static_cast<int64_t>(g_cl_cus) * per_cu;
  if (zg && grid > zslots) grid = zslots;
  if (grid > ntensor) grid = ntensor;
  hipLaunchKernelGGL(k_cluster_claim_reset, dim3(1), dim3(64), 0, stream, c.info);
  GLINT_LAUNCHED("k_cluster_claim_reset");
  if (zg)
    hipLaunchKernelGGL((k_cluster_als<TT, R, true>), dim3(static_cast<unsigned>(grid)), dim3(kClThreads), lds,
                       stream, c);
  else
    hipLaunchKernelGGL((k_cluster_als<TT, R, false>), dim3(static_cast<unsigned>(grid)), dim3(kClThreads), lds,
                       stream, c);
  GLINT_LAUNCHED("k_cluster_als");
  return GLINT_OK;
}

template <typename TT>
glint_status launch_cluster_als_r(const ClusterArgs& c, int64_t ntensor, bool run_mass, int64_t zslots,
                                  hipStream_t stream) {
  switch (c.R) {
    case 4: return launch_cluster_als<TT, 4>(c, ntensor, run_mass, zslots, stream);
    case 8: return launch_cluster_als<TT, 8>(c, ntensor, run_mass, zslots, stream);
    case 16: return launch_cluster_als<TT, 16>(c, ntensor, run_mass, zslots, stream);
    default: return launch_cluster_als<TT, 32>(c, ntensor, run_mass, zslots, stream);
  }
}

// Workspace of the map-driven calls: the texel bin windows, one angular
// block's tensor, the Z slots, the per-tensor counts and the scan's chunk sums.
struct MapWs {
  size_t bins, mass, sub, zws, counts, csum, total;
  int64_t zslots, zstride, nchunk;
};

MapWs map_workspace(const glint_ndf_desc* d, const ClShape& s, int R, glint_dtype dt) {
  MapWs w;
  const int K = glint_window_k(d);
  const size_t texels = static_cast<size_t>(d->nu) * d->nv;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t a = at;
    at += glint_round_up(bytes, 256);
    return a;
  };
  w.bins = take(sizeof(int32_t) * 2 * texels);
  w.mass = take(sizeof(double) * 2 * texels * (2 * K + 1));
  w.sub = take(glint_dtype_size(dt) * texels * d->nlevels * s.t * s.t);
  w.zslots = static_cast<int64_t>(kZSlotsPerCu) * g_cl_cus;
  w.zstride = static_cast<int64_t>(s.L) * (R + 1);
  w.zws = take(sizeof(double) * static_cast<size_t>(w.zslots * w.zstride));
  w.counts = take(sizeof(int32_t) * static_cast<size_t>(s.ntensor));
  w.nchunk = (s.ntensor + kScanChunk - 1) / kScanChunk;
  w.csum = take(sizeof(int64_t) * static_cast<size_t>(w.nchunk));
  w.total = at;
  return w;
}

// Arguments of the kernels for the tensor of angular block (zs, zt): T is
// that block's tensor (nbins = t, one block), its tensors numbered
// ((cu ncv + cv) nb + zs) nb + zt in the whole layout.
ClusterArgs map_args(const glint_ndf_desc* d, const glint_cluster_desc* cd, const ClShape& s, const void* sub,
                     int zs, int zt) {
  ClusterArgs c = {};
  c.T = sub; c.nu = d->nu; c.nv = d->nv; c.nl = d->nlevels; c.N = s.t;
  c.t = s.t; c.cs = cd->cs; c.ncv = s.ncv; c.nb = 1; c.L = s.L; c.R = cd->R;
  c.ntensor = static_cast<int>(s.ntensor / (static_cast<int64_t>(s.nb) * s.nb));
  c.tmul = static_cast<int64_t>(s.nb) * s.nb;
  c.tadd = static_cast<int64_t>(zs) * s.nb + zt;
  return c;
}

glint_status map_prologue(const glint_ndf_desc* desc, const glint_cluster_desc* cd, const float* nxy,
                          glint_dtype T_dtype, void* workspace, size_t workspace_bytes, ClShape* s, MapWs* w,
                          hipStream_t stream) {
  glint_status st = cluster_shape(desc, cd, s);
  if (st != GLINT_OK) return st;
  GLINT_SUPPORT(T_dtype == GLINT_F32 || T_dtype == GLINT_F64, "block tensors must be F32 or F64");
  GLINT_REQUIRE(nxy && workspace, "null pointer argument");
  GLINT_REQUIRE(glint_aligned(workspace, 256), "workspace must be 256-byte aligned");
  GLINT_SUPPORT(s->t * s->t % 4 == 0, "block side %d: t^2 must be a multiple of 4", s->t);
  if ((st = cl_device()) != GLINT_OK) return st;
  *w = map_workspace(desc, *s, cd->R, T_dtype);
  if (workspace_bytes < w->total)
    return glint_fail(GLINT_E_WORKSPACE, "workspace %zu < %zu bytes", workspace_bytes, w->total);
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  return glint_texel_bins(desc, nxy, reinterpret_cast<int32_t*>(ws + w->bins), reinterpret_cast<double*>(ws + w->mass),
                          stream);
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
  c.iters = iters; c.ntensor = static_cast<int>(s.ntensor); c.R = cd->R; c.seed = seed; c.X = X; c.Y = Y; c.Z = Z; c.blank = blank; c.info = info;
  c.tmul = 1; c.tadd = 0; c.zidx = nullptr; c.counts = nullptr; c.zws = nullptr; c.zws_stride = 0;
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_cluster_info_init, dim3(1), dim3(64), 0, stream, info);
  GLINT_LAUNCHED("k_cluster_info_init");
  if (T_dtype == GLINT_F64) return launch_cluster_als_r<double>(c, s.ntensor, true, 0, stream);
  return launch_cluster_als_r<float>(c, s.ntensor, true, 0, stream);
}

size_t glint_cluster_map_workspace(const glint_ndf_desc* desc, const glint_cluster_desc* cd, glint_dtype T_dtype) {
  ClShape s;
  if (cluster_shape(desc, cd, &s) != GLINT_OK || cl_device() != GLINT_OK) return 0;
  if (T_dtype != GLINT_F32 && T_dtype != GLINT_F64) return 0;
  return map_workspace(desc, s, cd->R, T_dtype).total;
}

glint_status glint_cluster_map_index(const glint_ndf_desc* desc, const glint_cluster_desc* cd, const float* nxy,
                                     glint_dtype T_dtype, int32_t* zidx, int64_t* zbase, int32_t* info,
                                     void* workspace, size_t workspace_bytes, hipStream_t stream) {
  ClShape s;
  MapWs w;
  GLINT_REQUIRE(zidx && zbase && info, "null pointer argument");
  glint_status st = map_prologue(desc, cd, nxy, T_dtype, workspace, workspace_bytes, &s, &w, stream);
  if (st != GLINT_OK) return st;
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  const int32_t* bins = reinterpret_cast<const int32_t*>(ws + w.bins);
  const double* mass = reinterpret_cast<const double*>(ws + w.mass);
  int32_t* counts = reinterpret_cast<int32_t*>(ws + w.counts);
  int64_t* csum = reinterpret_cast<int64_t*>(ws + w.csum);
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_cluster_info_init, dim3(1), dim3(64), 0, stream, info);
  GLINT_LAUNCHED("k_cluster_info_init");
  hipLaunchKernelGGL(k_fill_i32, dim3(static_cast<unsigned>((s.ntensor + 255) / 256)), dim3(256), 0, stream, counts,
                     s.ntensor, 0);
  GLINT_LAUNCHED("k_fill_i32");
  for (int zs = 0; zs < s.nb; ++zs)
    for (int zt = 0; zt < s.nb; ++zt) {
      if ((st = glint_build_window(desc, bins, mass, ws + w.sub, T_dtype, 1, zs * s.t, zt * s.t, s.t, stream)) !=
          GLINT_OK)
        return st;
      ClusterArgs c = map_args(desc, cd, s, ws + w.sub, zs, zt);
      c.zidx = zidx;
      c.counts = counts;
      c.info = info;
      glint_clear_launch_error();
      if (T_dtype == GLINT_F64)
        hipLaunchKernelGGL((k_cluster_mass<double>), dim3(static_cast<unsigned>(c.ntensor)), dim3(kMassThreads), 0,
                           stream, c);
      else
        hipLaunchKernelGGL((k_cluster_mass<float>), dim3(static_cast<unsigned>(c.ntensor)), dim3(kMassThreads), 0,
                           stream, c);
      GLINT_LAUNCHED("k_cluster_mass");
    }
  const unsigned nchunk = static_cast<unsigned>(w.nchunk);
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_scan_chunks, dim3(nchunk), dim3(kScanThreads), 0, stream, counts, s.ntensor, csum);
  GLINT_LAUNCHED("k_scan_chunks");
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, stream, csum, w.nchunk, zbase, s.ntensor, info);
  GLINT_LAUNCHED("k_scan_top");
  hipLaunchKernelGGL(k_scan_apply, dim3(nchunk), dim3(kScanThreads), 0, stream, counts, s.ntensor, csum, zbase);
  GLINT_LAUNCHED("k_scan_apply");
  hipLaunchKernelGGL(k_cluster_rows, dim3(static_cast<unsigned>((s.ntensor + 3) / 4)), dim3(256), 0, stream, zidx,
                     zbase, s.ntensor, s.L, info);
  GLINT_LAUNCHED("k_cluster_rows");
  return GLINT_OK;
}

glint_status glint_cp_als_clustered_map(const glint_ndf_desc* desc, const glint_cluster_desc* cd, const float* nxy,
                                        glint_dtype T_dtype, int32_t iters, uint64_t seed, const int32_t* zidx,
                                        float* X, float* Y, float* Z, uint8_t* blank, int32_t* info,
                                        void* workspace, size_t workspace_bytes, hipStream_t stream) {
  ClShape s;
  MapWs w;
  GLINT_REQUIRE(zidx && X && Y && Z && blank && info, "null pointer argument");
  GLINT_REQUIRE(iters >= 1, "iters must be >= 1");
  glint_status st = map_prologue(desc, cd, nxy, T_dtype, workspace, workspace_bytes, &s, &w, stream);
  if (st != GLINT_OK) return st;
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  const int32_t* bins = reinterpret_cast<const int32_t*>(ws + w.bins);
  const double* mass = reinterpret_cast<const double*>(ws + w.mass);
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_cluster_info_init, dim3(1), dim3(64), 0, stream, info);
  GLINT_LAUNCHED("k_cluster_info_init");
  for (int zs = 0; zs < s.nb; ++zs)
    for (int zt = 0; zt < s.nb; ++zt) {
      if ((st = glint_build_window(desc, bins, mass, ws + w.sub, T_dtype, 1, zs * s.t, zt * s.t, s.t, stream)) !=
          GLINT_OK)
        return st;
      ClusterArgs c = map_args(desc, cd, s, ws + w.sub, zs, zt);
      c.iters = iters; c.seed = seed; c.X = X; c.Y = Y; c.Z = Z; c.blank = blank; c.info = info;
      c.zidx = const_cast<int32_t*>(zidx);     // read only by the ALS kernel
      c.zws = reinterpret_cast<double*>(ws + w.zws);
      c.zws_stride = w.zstride;
      st = T_dtype == GLINT_F64 ? launch_cluster_als_r<double>(c, c.ntensor, false, w.zslots, stream)
                                : launch_cluster_als_r<float>(c, c.ntensor, false, w.zslots, stream);
      if (st != GLINT_OK) return st;
    }
  return GLINT_OK;
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
  GLINT_REQUIRE(f->dtype == GLINT_F32 || f->dtype == GLINT_BF16, "clustered tables must be F32 or BF16 (dtype %d)",
                f->dtype);
  if ((st = cl_device()) != GLINT_OK) return st;
  ClQueryArgs a;
  a.CX = f->CX; a.CY = f->CY; a.Z = f->Z; a.zidx = f->zidx;
  a.t = s.t; a.cs = f->cs; a.nu = f->nu; a.nv = f->nv; a.nl = f->nl; a.N = f->nbins;
  a.ncv = s.ncv; a.nb = s.nb; a.L = s.L; a.nq = nq; a.q = q; a.out = out;
  const int64_t waves = (nq + 63) / 64;
  int64_t blocks = (waves + 3) / 4;
  const int64_t cap = static_cast<int64_t>(g_cl_cus) * 8;
  if (blocks > cap) blocks = cap;
  glint_clear_launch_error();
  if (f->dtype == GLINT_BF16) {
    switch (f->R) {
      case 4: hipLaunchKernelGGL((k_query_clustered<uint16_t, 4>), dim3(blocks), dim3(kClQueryThreads), 0, stream, a); break;
      case 8: hipLaunchKernelGGL((k_query_clustered<uint16_t, 8>), dim3(blocks), dim3(kClQueryThreads), 0, stream, a); break;
      case 16: hipLaunchKernelGGL((k_query_clustered<uint16_t, 16>), dim3(blocks), dim3(kClQueryThreads), 0, stream, a); break;
      default: hipLaunchKernelGGL((k_query_clustered<uint16_t, 32>), dim3(blocks), dim3(kClQueryThreads), 0, stream, a); break;
    }
  } else {
    switch (f->R) {
      case 4: hipLaunchKernelGGL((k_query_clustered<float, 4>), dim3(blocks), dim3(kClQueryThreads), 0, stream, a); break;
      case 8: hipLaunchKernelGGL((k_query_clustered<float, 8>), dim3(blocks), dim3(kClQueryThreads), 0, stream, a); break;
      case 16: hipLaunchKernelGGL((k_query_clustered<float, 16>), dim3(blocks), dim3(kClQueryThreads), 0, stream, a); break;
      default: hipLaunchKernelGGL((k_query_clustered<float, 32>), dim3(blocks), dim3(kClQueryThreads), 0, stream, a); break;
    }
  }
  GLINT_LAUNCHED("k_query_clustered");
  return GLINT_OK;
}

glint_status glint_sample_clustered(const glint_clustered* f, int64_t n, const int32_t* uvl, const float* rnd,
                                    float* h, float* pdf, int32_t* bins, hipStream_t stream) {
  GLINT_REQUIRE(f != nullptr, "tables are NULL");
  glint_ndf_desc d;
  d.nu = f->nu; d.nv = f->nv; d.nlevels = f->nl; d.nbins = f->nbins; d.sigma = 0.01;
  glint_cluster_desc cd;
  cd.t = f->t; cd.cs = f->cs; cd.R = f->R;
  ClShape sh;
  glint_status st = cluster_shape(&d, &cd, &sh);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(f->t == sh.t, "block side must be min(t, nbins) = %d", sh.t);
  GLINT_REQUIRE((sh.t & (sh.t - 1)) == 0, "block side %d must be a power of two", sh.t);
  GLINT_REQUIRE(n >= 0, "n must be >= 0");
  if (n == 0) return GLINT_OK;
  GLINT_REQUIRE(f->CX && f->CY && f->Z && uvl && rnd && h && pdf && bins, "null pointer argument");
  if (f->dtype != GLINT_F32)
    return glint_fail(GLINT_E_UNSUPPORTED, "clustered sampling takes FP32 tables (dtype %d)", f->dtype);
  ClSampleArgs a;
  a.CX = static_cast<const float*>(f->CX); a.CY = static_cast<const float*>(f->CY);
  a.Z = static_cast<const float*>(f->Z); a.zidx = f->zidx;
  a.t = sh.t; a.cs = f->cs; a.nu = f->nu; a.nv = f->nv; a.nl = f->nl; a.N = f->nbins;
  a.ncv = sh.ncv; a.nb = sh.nb; a.L = sh.L;
  int levels = 0;
  while ((1 << levels) < sh.t) ++levels;
  a.levels = levels;
  a.n = n; a.uvl = uvl; a.rnd = rnd; a.h = h; a.pdf = pdf; a.bins = bins;
  const dim3 grid(static_cast<unsigned>((n + kClSampleThreads - 1) / kClSampleThreads));
  glint_clear_launch_error();
  switch (f->R) {
    case 4: hipLaunchKernelGGL(k_sample_clustered<4>, grid, dim3(kClSampleThreads), 0, stream, a); break;
    case 8: hipLaunchKernelGGL(k_sample_clustered<8>, grid, dim3(kClSampleThreads), 0, stream, a); break;
    case 16: hipLaunchKernelGGL(k_sample_clustered<16>, grid, dim3(kClSampleThreads), 0, stream, a); break;
    default: hipLaunchKernelGGL(k_sample_clustered<32>, grid, dim3(kClSampleThreads), 0, stream, a); break;
  }
  GLINT_LAUNCHED("k_sample_clustered");
  return GLINT_OK;
}

}  // extern "C"
