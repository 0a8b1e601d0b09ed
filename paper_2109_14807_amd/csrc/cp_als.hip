// CP decomposition of the NDF tensor by alternating least squares
// (Sec. 4.2, Eq. compress), entirely on the GPU with no host synchronisation.
//
// A sweep updates the factors in the order u, v, l, s, t; the update of mode n
// is A_n = M_n G^-1 with M_n the MTTKRP and G the Hadamard product of the other
// factors' Grams.  The five MTTKRPs of a sweep need only two passes over T:
//
//   Z pass  Z[cell][r] = sum_{s,t} T[cell][s,t] S[s][r] Tf[t][r]
//           (a GEMM ncells x N^2 times the N^2 x R Khatri-Rao block of S and
//           Tf, formed in registers), then
//           M_U[u] = sum_{v,l} V[v] L[l] Z[u,v,l],  M_V and M_L likewise with
//           the freshly updated factors (Z does not depend on U, V, L);
//   Y pass  Y[s,t][r] = sum_cell T[cell][s,t] U[u][r] V[v][r] L[l][r]
//           (a split-K GEMM N^2 x ncells times ncells x R), then
//           M_S[s] = sum_t Tf[t] Y[s,t],  M_T[t] = sum_s S_new[s] Y[s,t].
//
// Both passes run on the matrix cores (v_mfma_f64_16x16x4f64 for an FP64 T,
// v_mfma_f32_16x16x4f32 for an FP32 T) reading each T element once.  Grams,
// the Cholesky factorisation, the triangular solves, the column norms and the
// fit are FP64.  Every kernel reads a "done" flag first so that a sweep loop
// stopped by the tolerance costs only empty launches.
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "common.h"

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename AT>
struct Mfma;

// Both 16x16x4 shapes take A[i][k] from lane i + 16k and B[k][j] from lane
// j + 16k; the result D[i][j] sits in lane j + 16*(i/4) item i%4 for FP32 but
// in lane j + 16*(i%4) item i/4 for FP64 (measured on gfx950).  row(g, q) is
// the D row held in item q by the lanes of group g = lane/16.
template <>
struct Mfma<float> {
  typedef f32x4 acc_t;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int q) { return 4 * g + q; }
};

template <>
struct Mfma<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int q) { return g + 4 * q; }
};

// control block in the workspace
enum { CTRL_DONE = 0, CTRL_SWEEPS = 1, CTRL_FAILS = 2, CTRL_FAILNOW = 3, CTRL_N = 8 };

constexpr double kPivotRtol = 1e-13;
constexpr int kPad64 = 2;   // LDS row padding (elements) so 16 rows hit distinct banks
constexpr int kPad32 = 4;

// ---------------------------------------------------------------------------
// ||T||^2
// ---------------------------------------------------------------------------

// Clears the control words and the previous fit, and sets the column weights
// to 1: if no mode update succeeds, the initial factors are returned as given.
__global__ void k_als_init(int* __restrict__ ctrl, double* __restrict__ fitprev, double* __restrict__ lam, int R) {
  if (threadIdx.x < CTRL_N) ctrl[threadIdx.x] = 0;
  if (threadIdx.x == 0) fitprev[0] = 0.0;
  for (int r = threadIdx.x; r < R; r += blockDim.x) lam[r] = 1.0;
}

__global__ void k_fill_scalar(double* __restrict__ p, double v) { p[0] = v; }

// ||T||^2 from the per-wave partial sums of the first Z pass.
__global__ void k_sum_norm(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
  acc = glint_wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void k_ctrl_init(int* __restrict__ ctrl) {
  if (threadIdx.x < CTRL_N) ctrl[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// Z pass: Z[cell][r] = sum_k T[cell][k] W2[k][r],  W2[s*N+t][r] = S[s][r] Tf[t][r]
// A wave owns 16*ROWT cells and all R columns.  Lane (i = l%16, kk = l/16)
// loads VEC consecutive k of cell i; MFMA sub-step j takes k = k0 + kk*VEC + j.
// ---------------------------------------------------------------------------

template <typename TT, int R, int ROWT, int H>
__global__ __launch_bounds__(256) void k_mttkrp_z(const TT* __restrict__ T, int64_t ncells, int N,
                                                  const double* __restrict__ S,
                                                  const double* __restrict__ Tf,
                                                  TT* __restrict__ Z, double* __restrict__ sumsq,
                                                  const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  typedef Mfma<TT> M;
  typedef typename M::acc_t acc_t;
  typedef typename std::conditional<sizeof(TT) == 4, float4, double2>::type vec_t;
  constexpr int VEC = 16 / sizeof(TT);
  constexpr int CT = R / 16;
  constexpr int PAD = sizeof(TT) == 4 ? kPad32 : kPad64;
  extern __shared__ __align__(16) unsigned char smem[];
  TT* TfT = reinterpret_cast<TT*>(smem);   // [R][N + PAD]
  const int ld = N + PAD;
  TT* Ss = TfT + R * ld;                   // [N][R]
  for (int i = threadIdx.x; i < N * R; i += blockDim.x) {
    const int t = i / R, r = i - (i / R) * R;
    TfT[r * ld + t] = static_cast<TT>(Tf[i]);
    Ss[i] = static_cast<TT>(S[i]);
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int i16 = lane & 15;
  const int kk = lane >> 4;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t cell0 = wave * 16 * ROWT;
  if (cell0 >= ncells) return;
  const int64_t NN = static_cast<int64_t>(N) * N;

  acc_t acc[ROWT][CT];
#pragma unroll
  for (int rt = 0; rt < ROWT; ++rt)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[rt][c] = acc_t{};

  const TT* rowp[ROWT];
#pragma unroll
  for (int rt = 0; rt < ROWT; ++rt) {
    int64_t cell = cell0 + 16 * rt + i16;
    if (cell >= ncells) cell = ncells - 1;     // rows past the end load a valid row, never stored
    rowp[rt] = T + cell * NN + kk * VEC;   // + h*4*VEC for the second vector of a chunk
  }
  double ss = 0.0;                            // sum of squares of this lane's elements
  const bool own_rows = sumsq != nullptr;

  // flat loop over H*4*VEC-wide chunks of k = s*N + t: with H = 2 the four
  // lanes of a row read one whole 128-byte line per chunk (two 16-byte
  // vectors each, at kk*VEC and 4*VEC + kk*VEC); the next chunk's loads are
  // issued before this chunk's products
  constexpr int CW = H * 4 * VEC;            // k per chunk; N is a multiple
  const int chunks_per_row = N / CW;
  const int nchunks = N * chunks_per_row;
  vec_t nxt[ROWT][H];
#pragma unroll
  for (int rt = 0; rt < ROWT; ++rt)
#pragma unroll
    for (int h = 0; h < H; ++h) nxt[rt][h] = *reinterpret_cast<const vec_t*>(rowp[rt] + h * 4 * VEC);
  for (int ch = 0; ch < nchunks; ++ch) {
    const int s = ch / chunks_per_row;
    const int t0 = (ch - s * chunks_per_row) * CW;
    vec_t av[ROWT][H];
#pragma unroll
    for (int rt = 0; rt < ROWT; ++rt)
#pragma unroll
      for (int h = 0; h < H; ++h) av[rt][h] = nxt[rt][h];
    if (ch + 1 < nchunks) {
      const int s1 = (ch + 1) / chunks_per_row;
      const int64_t k1 = static_cast<int64_t>(s1) * N + (ch + 1 - s1 * chunks_per_row) * CW;
#pragma unroll
      for (int rt = 0; rt < ROWT; ++rt)
#pragma unroll
        for (int h = 0; h < H; ++h)
          nxt[rt][h] = *reinterpret_cast<const vec_t*>(rowp[rt] + k1 + h * 4 * VEC);
    }
    if (own_rows) {
#pragma unroll
      for (int rt = 0; rt < ROWT; ++rt)
        if (cell0 + 16 * rt + i16 < ncells)
#pragma unroll
          for (int h = 0; h < H; ++h)
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
              const double x = static_cast<double>(reinterpret_cast<const TT*>(&av[rt][h])[j]);
              ss += x * x;
            }
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const TT sv = Ss[s * R + 16 * c + i16];
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const vec_t tv =
            *reinterpret_cast<const vec_t*>(&TfT[(16 * c + i16) * ld + t0 + h * 4 * VEC + kk * VEC]);
        const TT* tvp = reinterpret_cast<const TT*>(&tv);
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
          const TT b = sv * tvp[j];
#pragma unroll
          for (int rt = 0; rt < ROWT; ++rt) {
            const TT a = reinterpret_cast<const TT*>(&av[rt][h])[j];
            acc[rt][c] = M::run(a, b, acc[rt][c]);
          }
        }
      }
    }
  }
  if (own_rows) {
    ss = glint_wave_sum(ss);
    if (lane == 0) sumsq[wave] = ss;
  }
  // D[m][n]: item q of this lane holds row M::row(lane/16, q), column lane%16
#pragma unroll
  for (int rt = 0; rt < ROWT; ++rt)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t cell = cell0 + 16 * rt + M::row(kk, q);
      if (cell < ncells) {
#pragma unroll
        for (int c = 0; c < CT; ++c) Z[cell * R + 16 * c + i16] = acc[rt][c][q];
      }
    }
}

// ---------------------------------------------------------------------------
// Y pass (split K over cells): Ypart[split][k][r] = sum_{cell in split} T[cell][k] C[cell][r],
// C[cell][r] = UV[u*nv+v][r] L[l][r] with UV = U*V precomputed per sweep.
// A wave owns 16*VEC rows k (VEC row tiles: tile j holds k = kb + m*VEC + j)
// and all R columns; it walks its split four cells per step (lane group kk
// takes cell c0 + kk), issuing the next step's loads before this step's MFMAs.
// ---------------------------------------------------------------------------

template <typename TT>
__global__ void k_uv_product(const double* __restrict__ U, const double* __restrict__ V, int nu,
                             int nv, int R, TT* __restrict__ UV, const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  const int64_t n = static_cast<int64_t>(nu) * nv * R;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int r = static_cast<int>(i % R);
    const int64_t uv = i / R;
    const int64_t u = uv / nv, v = uv - u * nv;
    UV[i] = static_cast<TT>(U[u * R + r] * V[v * R + r]);
  }
}

constexpr int kYWaves = 8;                   // waves per Y-pass block: adjacent k-slices of the same cells

template <typename TT, int R>
__global__ __launch_bounds__(64 * kYWaves) void k_mttkrp_y(const TT* __restrict__ T, int64_t ncells, int nl,
                                                  int N, const TT* __restrict__ UV,
                                                  const double* __restrict__ L,
                                                  int64_t cells_per_split, TT* __restrict__ Ypart,
                                                  const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  typedef Mfma<TT> M;
  typedef typename M::acc_t acc_t;
  typedef typename std::conditional<sizeof(TT) == 4, float4, double2>::type vec_t;
  constexpr int VEC = 16 / sizeof(TT);
  constexpr int CT = R / 16;
  // L rows padded by 16 elements: the four lane groups usually read four
  // consecutive levels, which then start on different LDS banks
  constexpr int LD = R + 16;
  __shared__ TT Lf[16 * LD];                // nl <= 16
  for (int i = threadIdx.x; i < nl * R; i += blockDim.x) Lf[(i / R) * LD + i % R] = static_cast<TT>(L[i]);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int i16 = lane & 15;
  const int kk = lane >> 4;
  const int w = threadIdx.x >> 6;
  const int64_t NN = static_cast<int64_t>(N) * N;
  const int64_t kb = (static_cast<int64_t>(blockIdx.x) * kYWaves + w) * 16 * VEC;
  if (kb >= NN) return;
  const int64_t c_begin = static_cast<int64_t>(blockIdx.y) * cells_per_split;
  int64_t c_end = c_begin + cells_per_split;
  if (c_end > ncells) c_end = ncells;

  acc_t acc[VEC][CT];
#pragma unroll
  for (int j = 0; j < VEC; ++j)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[j][c] = acc_t{};

  const TT* tb = T + kb + i16 * VEC;
  // Two quads per step: lane group kk takes cells c0 + kk and c0 + 4 + kk,
  // tracked as (uv, l) and advanced by 8 cells per step without division.
  const int adv_uv = 8 / nl, adv_l = 8 - (8 / nl) * nl;
  const int64_t last = c_end - 1;
  const int64_t uv_last = last / nl;
  int64_t cell[2] = {c_begin + kk, c_begin + 4 + kk};
  int64_t uv[2];
  int l[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    uv[h] = cell[h] / nl;
    l[h] = static_cast<int>(cell[h] - uv[h] * nl);
  }
  auto load = [&](int h, vec_t& av, TT* uvr) {
    const bool in = cell[h] < c_end;
    const int64_t cc = in ? cell[h] : last;       // clamped rows are loaded, then zeroed
    const int64_t uc = in ? uv[h] : uv_last;
    av = *reinterpret_cast<const vec_t*>(tb + cc * NN);
#pragma unroll
    for (int c = 0; c < CT; ++c) uvr[c] = UV[uc * R + 16 * c + i16];
  };
  vec_t av_n[2];
  TT uv_n[2][CT];
#pragma unroll
  for (int h = 0; h < 2; ++h) load(h, av_n[h], uv_n[h]);
  for (int64_t c0 = c_begin; c0 < c_end; c0 += 8) {
    vec_t av[2];
    TT bv[2][CT];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      av[h] = av_n[h];
      const TT keep = cell[h] < c_end ? TT(1) : TT(0);
      const TT* lrow = Lf + l[h] * LD + i16;
#pragma unroll
      for (int c = 0; c < CT; ++c) bv[h][c] = uv_n[h][c] * lrow[16 * c] * keep;
      cell[h] += 8;
      l[h] += adv_l;
      uv[h] += adv_uv;
      const bool wrap = l[h] >= nl;
      l[h] = wrap ? l[h] - nl : l[h];
      uv[h] = wrap ? uv[h] + 1 : uv[h];
    }
    if (c0 + 8 < c_end) {
#pragma unroll
      for (int h = 0; h < 2; ++h) load(h, av_n[h], uv_n[h]);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int j = 0; j < VEC; ++j) {
        const TT a = reinterpret_cast<const TT*>(&av[h])[j];
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[j][c] = M::run(a, bv[h][c], acc[j][c]);
      }
  }
  TT* out = Ypart + static_cast<int64_t>(blockIdx.y) * NN * R;
#pragma unroll
  for (int j = 0; j < VEC; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t k = kb + M::row(kk, q) * VEC + j;
#pragma unroll
      for (int c = 0; c < CT; ++c) out[k * R + 16 * c + i16] = acc[j][c][q];
    }
}

template <typename TT>
__global__ void k_reduce_splits(const TT* __restrict__ Ypart, int nsplit, int64_t n,
                                double* __restrict__ Y, const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double acc = 0.0;
    for (int p = 0; p < nsplit; ++p) acc += static_cast<double>(Ypart[p * n + i]);
    Y[i] = acc;
  }
}

// mode s (which=3): M[s][r] = sum_t F[t][r] Y[s*N+t][r];  mode t (which=4): M[t][r] = sum_s F[s][r] Y[s*N+t][r]
__global__ void k_mttkrp_st(const double* __restrict__ Y, const double* __restrict__ F, int N, int R,
                            int which, double* __restrict__ M, const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * R) return;
  const int a = idx / R, r = idx - (idx / R) * R;
  double acc = 0.0;
  for (int b = 0; b < N; ++b) {
    const int64_t k = which == 3 ? static_cast<int64_t>(a) * N + b : static_cast<int64_t>(b) * N + a;
    acc += F[b * R + r] * Y[k * R + r];
  }
  M[idx] = acc;
}

// ---------------------------------------------------------------------------
// Z reductions for modes u, v, l (FP64): a block takes one row of the mode
// and a chunk of one other index, reduces in registers and LDS, and adds R
// partial sums into M with FP64 atomics (M cleared first).
//   mode 0: M[u] += sum_{v in chunk, l} V[v] L[l] Z[u,v,l]      grid (nu, nv/kChunk)
//   mode 1: M[v] += sum_{u in chunk, l} U[u] L[l] Z[u,v,l]      grid (nv, nu/kChunk)
//   mode 2: M[l] += sum_{v in chunk}    U[u] V[v] Z[u,v,l]      grid (nu, nv/kChunk), all l
// ---------------------------------------------------------------------------

constexpr int kChunk = 16;

__global__ void k_zero(double* __restrict__ p, int64_t n, const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

template <typename TT, int MODE>
__global__ __launch_bounds__(256) void k_reduce_z(const TT* __restrict__ Z, int nu, int nv, int nl, int R,
                                                  const double* __restrict__ U,
                                                  const double* __restrict__ V,
                                                  const double* __restrict__ L,
                                                  double* __restrict__ M, const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  __shared__ double sh[16 * 256];
  const int r = threadIdx.x % R;
  const int parts = blockDim.x / R;
  const int p = threadIdx.x / R;
  const int row = blockIdx.x;                // u (modes 0, 2) or v (mode 1)
  const int c0 = blockIdx.y * kChunk;        // chunk of v (modes 0, 2) or u (mode 1)
  const int cn = min(kChunk, (MODE == 1 ? nu : nv) - c0);
  if (MODE == 2)
    for (int i = threadIdx.x; i < nl * 256; i += blockDim.x) sh[i] = 0.0;
  double acc = 0.0;
  if (MODE == 2) __syncthreads();
  if (p < parts) {
    for (int o = p; o < cn; o += parts) {    // one (u, v) pair: nl contiguous cells
      const int u = MODE == 1 ? c0 + o : row;
      const int v = MODE == 1 ? row : c0 + o;
      const TT* zc = Z + (static_cast<int64_t>(u) * nv + v) * nl * R + r;
      if (MODE == 0) {
        double t = 0.0;
        for (int l = 0; l < nl; ++l) t += L[l * R + r] * static_cast<double>(zc[l * R]);
        acc += V[static_cast<int64_t>(v) * R + r] * t;
      } else if (MODE == 1) {
        double t = 0.0;
        for (int l = 0; l < nl; ++l) t += L[l * R + r] * static_cast<double>(zc[l * R]);
        acc += U[static_cast<int64_t>(u) * R + r] * t;
      } else {
        const double w = U[static_cast<int64_t>(u) * R + r] * V[static_cast<int64_t>(v) * R + r];
        for (int l = 0; l < nl; ++l) sh[l * 256 + threadIdx.x] += w * static_cast<double>(zc[l * R]);
      }
    }
  }
  if (MODE != 2) sh[threadIdx.x] = acc;
  __syncthreads();
  const int nout = MODE == 2 ? nl : 1;
  for (int idx = threadIdx.x; idx < nout * R; idx += blockDim.x) {
    const int i = idx / R, rr = idx % R;
    double t = 0.0;
    for (int q = 0; q < parts; ++q) t += sh[i * 256 + q * R + rr];
    const int orow = MODE == 2 ? i : row;
    atomicAdd(&M[static_cast<int64_t>(orow) * R + rr], t);
  }
}

// ---------------------------------------------------------------------------
// Grams, Cholesky, solve, normalisation, fit (FP64)
// ---------------------------------------------------------------------------

__global__ void k_gram(const double* __restrict__ A, int rows, int R, double* __restrict__ G,
                       const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  const int i = blockIdx.y * 16 + threadIdx.y;
  const int j = blockIdx.x * 16 + threadIdx.x;
  if (i >= R || j >= R) return;
  double acc = 0.0;
  for (int k = 0; k < rows; ++k) acc += A[k * R + i] * A[k * R + j];
  G[i * R + j] = acc;
}

// One workgroup: G = Hadamard product of the Grams of the modes other than n,
// lower Cholesky factor in place (LDS), written as Lc and its transpose LcT.
// Cholesky factor of the Hadamard product of the four Grams other than mode n,
// held in registers: a GD x GD grid of threads, thread (a, b) owning the
// entries (a + GD e, b + GD f) of the lower triangle (f <= e).  Unscaled
// right-looking elimination: after step j the trailing block holds
// G - sum_{m<=j} c_m c_m^T / d_m with c_m the m-th column and d_m its pivot,
// and the factor L[i][j] = c_j[i] / sqrt(d_j) is formed at the end.  Column j
// goes through LDS (double-buffered, one barrier per column).  Breakdown: a
// pivot not above kPivotRtol times the original diagonal entry.
// side of the thread grid of k_cholesky (launched with its square as the block size):
// 16 x 16 up to rank 64 (fewer wavefronts per column barrier), else 32 x 32
constexpr int cholesky_grid(int R) { return R <= 16 ? R : (R <= 64 ? 16 : 32); }

template <int R>
__global__ __launch_bounds__(1024) void k_cholesky(const double* __restrict__ grams, int n,
                                                   double* __restrict__ Lc, double* __restrict__ LcT,
                                                   int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  constexpr int GD = cholesky_grid(R);
  constexpr int E = R / GD;
  constexpr int RR = R * R;
  __shared__ double col[2][R];
  __shared__ double diag0[R];
  const int t = threadIdx.x;
  const bool active = t < GD * GD;
  const int a = t / GD, b = t % GD;
  double g[E][E];
#pragma unroll
  for (int e = 0; e < E; ++e)
#pragma unroll
    for (int f = 0; f <= e; ++f) {
      g[e][f] = 0.0;
      if (active) {
        const int idx = (a + GD * e) * R + b + GD * f;
        double v = 1.0;
        for (int m = 0; m < 5; ++m)
          if (m != n) v *= grams[static_cast<int64_t>(m) * RR + idx];
        g[e][f] = v;
      }
    }
  if (active && a == b)
#pragma unroll
    for (int e = 0; e < E; ++e) diag0[a + GD * e] = g[e][e];
  __syncthreads();
  bool fail = false;
  for (int j = 0; j < R; ++j) {
    const int buf = j & 1;
    const int jb = j % GD, jf = j / GD;
    if (active && b == jb) {
#pragma unroll
      for (int e = 0; e < E; ++e)
#pragma unroll
        for (int f = 0; f <= e; ++f)
          if (f == jf && a + GD * e >= j) col[buf][a + GD * e] = g[e][f];
    }
    __syncthreads();
    const double d = col[buf][j];
    if (!(d > kPivotRtol * diag0[j])) {
      fail = true;
      break;
    }
    const double inv = 1.0 / d;
    if (active) {
      double ci[E], ck[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int i = a + GD * e, k = b + GD * e;
        ci[e] = i > j ? col[buf][i] : 0.0;
        ck[e] = k > j ? col[buf][k] : 0.0;
      }
#pragma unroll
      for (int e = 0; e < E; ++e)
#pragma unroll
        for (int f = 0; f <= e; ++f) {
          const int i = a + GD * e, k = b + GD * f;
          if (k > j && i >= k) g[e][f] -= ci[e] * ck[f] * inv;
        }
    }
  }
  if (t == 0) {
    ctrl[CTRL_FAILNOW] = fail ? 1 : 0;
    if (fail) ctrl[CTRL_FAILS] += 1;
  }
  if (fail) return;
  // sqrt of the final pivots through LDS (a second array: diag0 may still be
  // read by threads finishing the last step), then L and L^T
  __shared__ double dsq[R];
  if (active && a == b)
#pragma unroll
    for (int e = 0; e < E; ++e) dsq[a + GD * e] = sqrt(g[e][e]);
  __syncthreads();
  if (!active) return;
#pragma unroll
  for (int e = 0; e < E; ++e)
#pragma unroll
    for (int f = 0; f < E; ++f) {
      const int i = a + GD * e, k = b + GD * f;
      double x = 0.0;
      if (f <= e) {
        if (k < i) x = g[e][f] / dsq[k];
        else if (k == i) x = dsq[i];
      }
      Lc[i * R + k] = x;
      LcT[k * R + i] = x;
    }
}

// Fallback of a failed Cholesky (reading R4): the pseudo-inverse of the
// Hadamard Gram G of mode n through its eigendecomposition,
//   G+ = Q diag(1/w_i for w_i > 1e-12 w_max, else 0) Q^T,
// the eigenpairs by cyclic Jacobi rotations in one workgroup.  Each round
// rotates R/2 disjoint index pairs at once (round-robin order: index 0 stays,
// the others move one place per round, so R - 1 rounds meet every pair
// once); a pair is rotated when |a_pq| > 1e-15 sqrt|a_pp a_qq| (the
// symmetric 2x2 Schur rotation that zeroes a_pq); sweeps stop when one
// rotates nothing, at most kJacobiSweeps.  Every 2x2 block (pair k rows,
// pair m columns) of A = J^T A J is owned by one thread per round, and
// Q = Q J.  A and Q live in the R x R Cholesky buffers (Lc, LcT), unused when
// the factorisation failed; G+ is left in Lc for k_solve.  Runs only after a
// failed factorisation (ctrl[CTRL_FAILNOW]).
constexpr int kJacobiSweeps = 40;

__device__ __forceinline__ int jacobi_player(int j, int round, int R) {
  return j == 0 ? 0 : 1 + (j - 1 + round) % (R - 1);
}

template <int R>
__global__ __launch_bounds__(1024) void k_eigh_pinv(const double* __restrict__ grams, int n, double* A,
                                                    double* Q, const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE] || !ctrl[CTRL_FAILNOW]) return;
  constexpr int H = R / 2;
  constexpr int RR = R * R;
  __shared__ double cs[H], sn[H], wv[R];
  __shared__ int pp[H], qq[H], act[H];
  __shared__ int rotated;
  __shared__ double wmax_s;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int idx = tid; idx < RR; idx += nt) {
    double v = 1.0;
    for (int m = 0; m < 5; ++m)
      if (m != n) v *= grams[static_cast<int64_t>(m) * RR + idx];
    A[idx] = v;
    Q[idx] = (idx / R == idx % R) ? 1.0 : 0.0;
  }
  __threadfence_block();
  __syncthreads();
  for (int sweep = 0; sweep < kJacobiSweeps; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < R - 1; ++round) {
      if (tid < H) {
        const int p = jacobi_player(tid, round, R), q = jacobi_player(R - 1 - tid, round, R);
        const double apq = A[p * R + q], app = A[p * R + p], aqq = A[q * R + q];
        double c = 1.0, s = 0.0;
        int a = 0;
        if (fabs(apq) > 1e-15 * sqrt(fabs(app * aqq)) && fabs(apq) > 1e-300) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
          a = 1;
          rotated = 1;
        }
        cs[tid] = c;
        sn[tid] = s;
        pp[tid] = p;
        qq[tid] = q;
        act[tid] = a;
      }
      __syncthreads();
      for (int b = tid; b < H * H; b += nt) {
        const int k = b / H, m = b % H;
        const int pk = pp[k], qk = qq[k], pm = pp[m], qm = qq[m];
        const double ck = cs[k], sk = sn[k], cm = cs[m], sm = sn[m];
        const double a00 = A[pk * R + pm], a01 = A[pk * R + qm], a10 = A[qk * R + pm], a11 = A[qk * R + qm];
        const double r00 = ck * a00 - sk * a10, r01 = ck * a01 - sk * a11;
        const double r10 = sk * a00 + ck * a10, r11 = sk * a01 + ck * a11;
        double n01 = sm * r00 + cm * r01, n10 = cm * r10 - sm * r11;
        if (k == m && act[k]) n01 = n10 = 0.0;
        A[pk * R + pm] = cm * r00 - sm * r01;
        A[pk * R + qm] = n01;
        A[qk * R + pm] = n10;
        A[qk * R + qm] = sm * r10 + cm * r11;
      }
      for (int b = tid; b < R * H; b += nt) {
        const int i = b / H, m = b % H;
        const int p = pp[m], q = qq[m];
        const double c = cs[m], s = sn[m];
        const double qp = Q[i * R + p], qv = Q[i * R + q];
        Q[i * R + p] = c * qp - s * qv;
        Q[i * R + q] = s * qp + c * qv;
      }
      __threadfence_block();
      __syncthreads();
    }
    // every thread reads the flag before thread 0 may clear it for the next sweep
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
  for (int i = tid; i < R; i += nt) wv[i] = A[i * R + i];
  __syncthreads();
  if (tid == 0) {
    double wm = wv[0];
    for (int i = 1; i < R; ++i) wm = fmax(wm, wv[i]);
    wmax_s = wm;
  }
  __syncthreads();
  const double cut = 1e-12 * fmax(wmax_s, 0.0);
  for (int i = tid; i < R; i += nt) wv[i] = wv[i] > cut ? 1.0 / wv[i] : 0.0;
  __syncthreads();
  for (int idx = tid; idx < RR; idx += nt) {
    const int i = idx / R, j = idx % R;
    double acc = 0.0;
    for (int k = 0; k < R; ++k) acc += Q[i * R + k] * wv[k] * Q[j * R + k];
    A[idx] = acc;
  }
}

// One wave per row: x = m G^-1 with G = Lc Lc^T (forward then back
// substitution).  For R <= 128 the factor is staged once per block in LDS
// with row stride R + 1 (dynamic LDS of solve_lds_bytes(R)), so both the
// column walk of the forward pass and the row walk of the back pass are
// served without bank conflicts; larger ranks read it from global memory.
template <int R>
constexpr size_t solve_lds_bytes() {
  return R <= 128 ? sizeof(double) * R * (R + 1) : 0;
}

template <int R>
__global__ __launch_bounds__(1024) void k_solve(const double* __restrict__ M, int rows,
                                               const double* Lc, const double* LcT,
                                               double* __restrict__ A, const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  constexpr int E = (R + 63) / 64;
  constexpr bool kStage = R <= 128;
  constexpr int LD = kStage ? R + 1 : R;
  extern __shared__ __align__(16) double sL[];
  if (ctrl[CTRL_FAILNOW]) {
    // the factorisation failed: x = m G+ with the pseudo-inverse k_eigh_pinv left in Lc
    const int lane = threadIdx.x & 63;
    const int row = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (row >= rows) return;
    double w[E];
#pragma unroll
    for (int t = 0; t < E; ++t) w[t] = 0.0;
    for (int j = 0; j < R; ++j) {
      const double mj = M[static_cast<int64_t>(row) * R + j];
#pragma unroll
      for (int t = 0; t < E; ++t) {
        const int e = lane + 64 * t;
        if (e < R) w[t] += mj * Lc[j * R + e];
      }
    }
#pragma unroll
    for (int t = 0; t < E; ++t) {
      const int e = lane + 64 * t;
      if (e < R) A[static_cast<int64_t>(row) * R + e] = w[t];
    }
    return;
  }
  const double* Lf;   // L[i][k] at Lf[i * LD + k]
  if constexpr (kStage) {
    for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) {
      const int i = idx / R, k = idx % R;
      if (k <= i) sL[i * LD + k] = Lc[idx];
    }
    __syncthreads();
    Lf = sL;
  } else {
    Lf = Lc;
  }
  const int lane = threadIdx.x & 63;
  const int row = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (row >= rows) return;
  double w[E];
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const int e = lane + 64 * t;
    w[t] = e < R ? M[static_cast<int64_t>(row) * R + e] : 0.0;
  }
  // forward: L y = m (column j of L: L[e][j], e > j)
  for (int j = 0; j < R; ++j) {
    const int slot = j >> 6, owner = j & 63;
    double wj = 0.0;
#pragma unroll
    for (int t = 0; t < E; ++t)
      if (t == slot) wj = w[t];
    const double yj = __shfl(wj, owner) / Lf[j * LD + j];
#pragma unroll
    for (int t = 0; t < E; ++t) {
      const int e = lane + 64 * t;
      if (e == j) w[t] = yj;
      else if (e > j && e < R) w[t] -= (kStage ? Lf[e * LD + j] : LcT[j * R + e]) * yj;
    }
  }
  // back: L^T x = y (row j of L: L[j][e], e < j)
  for (int j = R - 1; j >= 0; --j) {
    const int slot = j >> 6, owner = j & 63;
    double wj = 0.0;
#pragma unroll
    for (int t = 0; t < E; ++t)
      if (t == slot) wj = w[t];
    const double xj = __shfl(wj, owner) / Lf[j * LD + j];
#pragma unroll
    for (int t = 0; t < E; ++t) {
      const int e = lane + 64 * t;
      if (e == j) w[t] = xj;
      else if (e < j) w[t] -= Lf[j * LD + e] * xj;
    }
  }
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const int e = lane + 64 * t;
    if (e < R) A[static_cast<int64_t>(row) * R + e] = w[t];
  }
}

// One workgroup: column norms lambda, unit columns, and the new Gram A^T A.
__global__ __launch_bounds__(1024) void k_normalize_gram(double* __restrict__ A, int rows, int R,
                                                         double* __restrict__ lam, double* __restrict__ G,
                                                         const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  __shared__ double sh[1024];
  __shared__ double lr[256];
  const int r = threadIdx.x % R;
  const int parts = blockDim.x / R;
  const int p = threadIdx.x / R;
  double s2 = 0.0;
  if (p < parts)
    for (int i = p; i < rows; i += parts) {
      const double x = A[static_cast<int64_t>(i) * R + r];
      s2 += x * x;
    }
  sh[threadIdx.x] = s2;
  __syncthreads();
  if (threadIdx.x < R) {
    double t = 0.0;
    for (int q = 0; q < parts; ++q) t += sh[q * R + threadIdx.x];
    const double nrm = sqrt(t);
    lam[threadIdx.x] = nrm;
    lr[threadIdx.x] = nrm;
  }
  __syncthreads();
  const int64_t n = static_cast<int64_t>(rows) * R;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double nrm = lr[i % R];
    if (nrm > 0.0) A[i] /= nrm;
  }
  if (G == nullptr) return;
  __syncthreads();
  // Gram in row tiles staged through LDS (tile of kGramRows x R doubles)
  constexpr int kGramRows = 4096 / 128;      // 32 rows of up to 128 columns = 32 KB
  __shared__ double tile[kGramRows * 128];
  constexpr int kMaxPer = 16;                // R*R / 1024 <= 16 for R <= 128
  double acc[kMaxPer];
#pragma unroll
  for (int e = 0; e < kMaxPer; ++e) acc[e] = 0.0;
  for (int k0 = 0; k0 < rows; k0 += kGramRows) {
    const int kn = min(kGramRows, rows - k0);
    for (int i = threadIdx.x; i < kn * R; i += blockDim.x) tile[i] = A[static_cast<int64_t>(k0) * R + i];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kMaxPer; ++e) {
      const int idx = threadIdx.x + e * 1024;
      if (idx < R * R) {
        const int i = idx / R, j = idx % R;
        double t = 0.0;
        for (int k = 0; k < kn; ++k) t += tile[k * R + i] * tile[k * R + j];
        acc[e] += t;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < kMaxPer; ++e) {
    const int idx = threadIdx.x + e * 1024;
    if (idx < R * R) G[idx] = acc[e];
  }
}

// fit = 1 - ||T - T^|| / ||T|| after the t update of sweep `it`.
__global__ __launch_bounds__(256) void k_fit(const double* __restrict__ grams, const double* __restrict__ lam,
                                             const double* __restrict__ Mt, const double* __restrict__ At,
                                             int N, int R, const double* __restrict__ normT2, int it,
                                             double tol, double* __restrict__ fit_hist,
                                             double* __restrict__ fitprev, int* __restrict__ ctrl) {
  __shared__ double sh[8];
  if (ctrl[CTRL_DONE]) {
    if (threadIdx.x == 0) fit_hist[it] = fitprev[0];
    return;
  }
  double inner = 0.0, hat = 0.0;
  for (int idx = threadIdx.x; idx < N * R; idx += blockDim.x) {
    const int r = idx % R;
    inner += lam[r] * Mt[idx] * At[idx];
  }
  const int RR = R * R;
  for (int idx = threadIdx.x; idx < RR; idx += blockDim.x) {
    double g = lam[idx / R] * lam[idx % R];
    for (int m = 0; m < 5; ++m) g *= grams[static_cast<int64_t>(m) * RR + idx];
    hat += g;
  }
  inner = glint_wave_sum(inner);
  hat = glint_wave_sum(hat);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[w] = inner;
    sh[4 + w] = hat;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double in = sh[0] + sh[1] + sh[2] + sh[3];
    const double nh = sh[4] + sh[5] + sh[6] + sh[7];
    const double t2 = normT2[0];
    double res2 = t2 - 2.0 * in + nh;
    if (res2 < 0.0) res2 = 0.0;
    const double fit = t2 > 0.0 ? 1.0 - sqrt(res2) / sqrt(t2) : __builtin_nan("");
    fit_hist[it] = fit;
    ctrl[CTRL_SWEEPS] = it + 1;
    if (tol > 0.0 && it > 0 && fabs(fit - fitprev[0]) < tol) ctrl[CTRL_DONE] = 1;
    fitprev[0] = fit;
  }
}

__global__ void k_absorb(double* __restrict__ L, int nl, int R, const double* __restrict__ lam,
                         const int* __restrict__ ctrl, int* __restrict__ info) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < nl * R) L[idx] *= lam[idx % R];
  if (idx == 0 && info) {
    info[0] = ctrl[CTRL_SWEEPS];
    info[1] = ctrl[CTRL_FAILS];
    info[2] = 0;
    info[3] = 0;
  }
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------

struct AlsLayout {
  size_t z, ypart, y, uv, m, grams, lc, lct, lam, sumsq, scal, ctrl, total;
  int nsplit;
  int64_t cells_per_split;
  int sumsq_blocks;
};

bool als_layout(const glint_ndf_desc* d, int R, size_t elt, AlsLayout* L) {
  const int64_t ncells = static_cast<int64_t>(d->nu) * d->nv * d->nlevels;
  const int64_t NN = static_cast<int64_t>(d->nbins) * d->nbins;
  const int VEC = static_cast<int>(16 / elt);
  const int64_t kblocks = (NN + 16 * kYWaves * VEC - 1) / (16 * kYWaves * VEC);
  int64_t nsplit = 1024 / (kblocks > 0 ? kblocks : 1);
  if (nsplit < 1) nsplit = 1;
  if (nsplit > (ncells + 63) / 64) nsplit = (ncells + 63) / 64;
  if (nsplit < 1) nsplit = 1;
  int64_t cps = (ncells + nsplit - 1) / nsplit;
  cps = (cps + 7) / 8 * 8;
  nsplit = (ncells + cps - 1) / cps;
  L->nsplit = static_cast<int>(nsplit);
  L->cells_per_split = cps;
  L->sumsq_blocks = static_cast<int>((ncells + 15) / 16);   // one partial per Z-pass wave (16*ROWT >= 16 cells)
  const int maxrows = std::max(std::max(d->nu, d->nv), std::max(d->nlevels, d->nbins));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += glint_round_up(bytes, 256);
    return at;
  };
  L->z = take(elt * ncells * R);
  L->ypart = take(elt * nsplit * NN * R);
  L->y = take(sizeof(double) * NN * R);
  L->uv = take(elt * static_cast<size_t>(d->nu) * d->nv * R);
  L->m = take(sizeof(double) * maxrows * R);
  L->grams = take(sizeof(double) * 5 * R * R);
  L->lc = take(sizeof(double) * R * R);
  L->lct = take(sizeof(double) * R * R);
  L->lam = take(sizeof(double) * R);
  L->sumsq = take(sizeof(double) * L->sumsq_blocks);
  L->scal = take(sizeof(double) * 4);
  L->ctrl = take(sizeof(int) * CTRL_N);
  L->total = off;
  return true;
}

template <typename TT>
glint_status reduce_z(int mode, const TT* Z, int nu, int nv, int nl, int R, const double* const F[5],
                      double* M, const int* ctrl, hipStream_t stream) {
  const int rows = mode == 0 ? nu : (mode == 1 ? nv : nl);
  hipLaunchKernelGGL(k_zero, dim3((rows * R + 255) / 256), dim3(256), 0, stream, M,
                     static_cast<int64_t>(rows) * R, ctrl);
  const dim3 grid(mode == 1 ? nv : nu, ((mode == 1 ? nu : nv) + kChunk - 1) / kChunk);
  if (mode == 0)
    hipLaunchKernelGGL((k_reduce_z<TT, 0>), grid, dim3(256), 0, stream, Z, nu, nv, nl, R, F[0], F[1], F[2], M, ctrl);
  else if (mode == 1)
    hipLaunchKernelGGL((k_reduce_z<TT, 1>), grid, dim3(256), 0, stream, Z, nu, nv, nl, R, F[0], F[1], F[2], M, ctrl);
  else
    hipLaunchKernelGGL((k_reduce_z<TT, 2>), grid, dim3(256), 0, stream, Z, nu, nv, nl, R, F[0], F[1], F[2], M, ctrl);
  GLINT_LAUNCHED("k_reduce_z");
  return GLINT_OK;
}

template <typename TT, int R>
glint_status run_als(const glint_ndf_desc* d, const TT* T, int iters, double tol, double* F[5],
                     double* fit_hist, int32_t* info, unsigned char* ws, const AlsLayout& Lo,
                     hipStream_t stream) {
  const int nu = d->nu, nv = d->nv, nl = d->nlevels, N = d->nbins;
  const int rows[5] = {nu, nv, nl, N, N};
  const int64_t ncells = static_cast<int64_t>(nu) * nv * nl;
  const int64_t NN = static_cast<int64_t>(N) * N;
  TT* Z = reinterpret_cast<TT*>(ws + Lo.z);
  TT* Yp = reinterpret_cast<TT*>(ws + Lo.ypart);
  double* Y = reinterpret_cast<double*>(ws + Lo.y);
  double* Mb = reinterpret_cast<double*>(ws + Lo.m);
  double* grams = reinterpret_cast<double*>(ws + Lo.grams);
  double* Lc = reinterpret_cast<double*>(ws + Lo.lc);
  double* LcT = reinterpret_cast<double*>(ws + Lo.lct);
  double* lam = reinterpret_cast<double*>(ws + Lo.lam);
  double* sumsq = reinterpret_cast<double*>(ws + Lo.sumsq);
  double* scal = reinterpret_cast<double*>(ws + Lo.scal);   // [0] ||T||^2, [1] previous fit
  int* ctrl = reinterpret_cast<int*>(ws + Lo.ctrl);

  constexpr int ROWT = R <= 64 ? 2 : 1;
  constexpr int PAD = sizeof(TT) == 4 ? kPad32 : kPad64;
  const size_t z_lds = sizeof(TT) * R * (2 * N + PAD);
  TT* UVt = reinterpret_cast<TT*>(ws + Lo.uv);

  glint_clear_launch_error();
  hipLaunchKernelGGL(k_als_init, dim3(1), dim3(64), 0, stream, ctrl, scal + 1, lam, R);
  GLINT_LAUNCHED("k_als_init");
  const dim3 gblk(16, 16), ggrid((R + 15) / 16, (R + 15) / 16);
  for (int m = 0; m < 5; ++m)
    hipLaunchKernelGGL(k_gram, ggrid, gblk, 0, stream, F[m], rows[m], R, grams + m * R * R, ctrl);
  GLINT_LAUNCHED("k_gram");

  auto update = [&](int n) -> glint_status {
    hipLaunchKernelGGL((k_cholesky<R>), dim3(1), dim3(cholesky_grid(R) * cholesky_grid(R)), 0, stream, grams, n, Lc,
                       LcT, ctrl);
    GLINT_LAUNCHED("k_cholesky");
    hipLaunchKernelGGL((k_eigh_pinv<R>), dim3(1), dim3(1024), 0, stream, grams, n, Lc, LcT, ctrl);
    GLINT_LAUNCHED("k_eigh_pinv");
    const int rws = rows[n];
    hipLaunchKernelGGL((k_solve<R>), dim3((rws + 15) / 16), dim3(1024), solve_lds_bytes<R>(), stream, Mb, rws, Lc,
                       LcT, F[n], ctrl);
    GLINT_LAUNCHED("k_solve");
    hipLaunchKernelGGL(k_normalize_gram, dim3(1), dim3(1024), 0, stream, F[n], rws, R, lam,
                       grams + n * R * R, ctrl);
    GLINT_LAUNCHED("k_normalize_gram");
    return GLINT_OK;
  };

  const int64_t zwaves = (ncells + 16 * ROWT - 1) / (16 * ROWT);
  const unsigned zblocks = static_cast<unsigned>((zwaves + 3) / 4);
  const int VEC = 16 / sizeof(TT);
  const unsigned yblocks = static_cast<unsigned>((NN + 16 * kYWaves * VEC - 1) / (16 * kYWaves * VEC));
  for (int it = 0; it < iters; ++it) {
    if (N >= 8 * VEC)
      hipLaunchKernelGGL((k_mttkrp_z<TT, R, ROWT, 2>), dim3(zblocks), dim3(256), z_lds, stream, T, ncells,
                         N, F[3], F[4], Z, it == 0 ? sumsq : nullptr, ctrl);
    else
      hipLaunchKernelGGL((k_mttkrp_z<TT, R, ROWT, 1>), dim3(zblocks), dim3(256), z_lds, stream, T, ncells,
                         N, F[3], F[4], Z, it == 0 ? sumsq : nullptr, ctrl);
    GLINT_LAUNCHED("k_mttkrp_z");
    if (it == 0) {
      hipLaunchKernelGGL(k_sum_norm, dim3(1), dim3(256), 0, stream, sumsq, static_cast<int>(zwaves), scal);
      GLINT_LAUNCHED("k_sum_norm");
    }
    glint_status st = reduce_z<TT>(0, Z, nu, nv, nl, R, F, Mb, ctrl, stream);
    if (st != GLINT_OK || (st = update(0)) != GLINT_OK) return st;
    if ((st = reduce_z<TT>(1, Z, nu, nv, nl, R, F, Mb, ctrl, stream)) != GLINT_OK) return st;
    if ((st = update(1)) != GLINT_OK) return st;
    if ((st = reduce_z<TT>(2, Z, nu, nv, nl, R, F, Mb, ctrl, stream)) != GLINT_OK) return st;
    if ((st = update(2)) != GLINT_OK) return st;
    hipLaunchKernelGGL(k_uv_product<TT>, dim3(2048), dim3(256), 0, stream, F[0], F[1], nu, nv, R, UVt, ctrl);
    hipLaunchKernelGGL((k_mttkrp_y<TT, R>), dim3(yblocks, Lo.nsplit), dim3(64 * kYWaves), 0, stream, T, ncells, nl, N,
                       UVt, F[2], Lo.cells_per_split, Yp, ctrl);
    GLINT_LAUNCHED("k_mttkrp_y");
    hipLaunchKernelGGL(k_reduce_splits<TT>, dim3(static_cast<unsigned>(std::min<int64_t>((NN * R + 255) / 256, 4096))),
                       dim3(256), 0, stream, Yp, Lo.nsplit, NN * R, Y, ctrl);
    GLINT_LAUNCHED("k_reduce_splits");
    hipLaunchKernelGGL(k_mttkrp_st, dim3((N * R + 255) / 256), dim3(256), 0, stream, Y, F[4], N, R, 3, Mb, ctrl);
    GLINT_LAUNCHED("k_mttkrp_st");
    if ((st = update(3)) != GLINT_OK) return st;
    hipLaunchKernelGGL(k_mttkrp_st, dim3((N * R + 255) / 256), dim3(256), 0, stream, Y, F[3], N, R, 4, Mb, ctrl);
    GLINT_LAUNCHED("k_mttkrp_st");
    if ((st = update(4)) != GLINT_OK) return st;
    hipLaunchKernelGGL(k_fit, dim3(1), dim3(256), 0, stream, grams, lam, Mb, F[4], N, R, scal, it, tol,
                       fit_hist, scal + 1, ctrl);
    GLINT_LAUNCHED("k_fit");
  }
  hipLaunchKernelGGL(k_absorb, dim3((nl * R + 255) / 256), dim3(256), 0, stream, F[2], nl, R, lam, ctrl, info);
  GLINT_LAUNCHED("k_absorb");
  return GLINT_OK;
}

template <typename TT, int R>
glint_status run_mttkrp(const glint_ndf_desc* d, const TT* T, int mode, const double* const F[5],
                        double* M, unsigned char* ws, const AlsLayout& Lo, hipStream_t stream) {
  const int nu = d->nu, nv = d->nv, nl = d->nlevels, N = d->nbins;
  const int64_t ncells = static_cast<int64_t>(nu) * nv * nl;
  const int64_t NN = static_cast<int64_t>(N) * N;
  TT* Z = reinterpret_cast<TT*>(ws + Lo.z);
  TT* Yp = reinterpret_cast<TT*>(ws + Lo.ypart);
  double* Y = reinterpret_cast<double*>(ws + Lo.y);
  int* ctrl = reinterpret_cast<int*>(ws + Lo.ctrl);
  constexpr int ROWT = R <= 64 ? 2 : 1;
  constexpr int PAD = sizeof(TT) == 4 ? kPad32 : kPad64;
  const int VEC = 16 / sizeof(TT);
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, stream, ctrl);
  GLINT_LAUNCHED("k_ctrl_init");
  if (mode <= 2) {
    const int64_t zwaves = (ncells + 16 * ROWT - 1) / (16 * ROWT);
    if (N >= 8 * VEC)
      hipLaunchKernelGGL((k_mttkrp_z<TT, R, ROWT, 2>), dim3(static_cast<unsigned>((zwaves + 3) / 4)), dim3(256),
                         sizeof(TT) * R * (2 * N + PAD), stream, T, ncells, N, F[3], F[4], Z, nullptr, ctrl);
    else
      hipLaunchKernelGGL((k_mttkrp_z<TT, R, ROWT, 1>), dim3(static_cast<unsigned>((zwaves + 3) / 4)), dim3(256),
                         sizeof(TT) * R * (2 * N + PAD), stream, T, ncells, N, F[3], F[4], Z, nullptr, ctrl);
    GLINT_LAUNCHED("k_mttkrp_z");
    glint_status st = reduce_z<TT>(mode, Z, nu, nv, nl, R, F, M, ctrl, stream);
    if (st != GLINT_OK) return st;
  } else {
    const unsigned yblocks = static_cast<unsigned>((NN + 16 * kYWaves * VEC - 1) / (16 * kYWaves * VEC));
    TT* UVt = reinterpret_cast<TT*>(ws + Lo.uv);
    hipLaunchKernelGGL(k_uv_product<TT>, dim3(2048), dim3(256), 0, stream, F[0], F[1], nu, nv, R, UVt, ctrl);
    hipLaunchKernelGGL((k_mttkrp_y<TT, R>), dim3(yblocks, Lo.nsplit), dim3(64 * kYWaves), 0, stream, T, ncells, nl, N,
                       UVt, F[2], Lo.cells_per_split, Yp, ctrl);
    GLINT_LAUNCHED("k_mttkrp_y");
    hipLaunchKernelGGL(k_reduce_splits<TT>, dim3(static_cast<unsigned>(std::min<int64_t>((NN * R + 255) / 256, 4096))),
                       dim3(256), 0, stream, Yp, Lo.nsplit, NN * R, Y, ctrl);
    hipLaunchKernelGGL(k_mttkrp_st, dim3((N * R + 255) / 256), dim3(256), 0, stream, Y,
                       mode == 3 ? F[4] : F[3], N, R, mode, M, ctrl);
    GLINT_LAUNCHED("k_mttkrp_st");
  }
  return GLINT_OK;
}

glint_status check_als_args(const glint_ndf_desc* desc, const void* T, glint_dtype T_dtype, int32_t R,
                            void* workspace, size_t workspace_bytes, AlsLayout* Lo) {
  glint_status st = glint_check_desc(desc);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(T && workspace, "null pointer argument");
  GLINT_SUPPORT(R == 16 || R == 32 || R == 64 || R == 128, "rank %d not in {16,32,64,128}", R);
  GLINT_SUPPORT(T_dtype == GLINT_F64 || T_dtype == GLINT_F32, "T dtype must be F64 or F32");
  GLINT_SUPPORT(desc->nbins >= 16, "ALS needs nbins >= 16");
  GLINT_REQUIRE(glint_aligned(T, 16) && glint_aligned(workspace, 256),
                "T must be 16-byte and workspace 256-byte aligned");
  als_layout(desc, R, glint_dtype_size(T_dtype), Lo);
  if (workspace_bytes < Lo->total)
    return glint_fail(GLINT_E_WORKSPACE, "workspace %zu < %zu bytes", workspace_bytes, Lo->total);
  int dev = 0, max_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return glint_fail(GLINT_E_HIP, "hipDeviceGetAttribute failed");
  const size_t pad = T_dtype == GLINT_F32 ? kPad32 : kPad64;
  if (static_cast<size_t>(max_lds) < glint_dtype_size(T_dtype) * R * (2 * desc->nbins + pad))
    return glint_fail(GLINT_E_UNSUPPORTED, "rank %d x %d bins factor block does not fit in LDS", R,
                      desc->nbins);
  return GLINT_OK;
}


// ===========================================================================
// Texel-space MTTKRP and ALS: the same contractions for the tensor built from
// per-texel bin windows (T[u,v,l] = k^-2 sum_{footprint} m_s (x) m_t), evaluated
// without forming T, so maps whose tensor exceeds HBM can be decomposed.
// With gs = S contracted with each texel's s-window, gt likewise for t,
// P = gs * gt and Ubar_l[x] = sum_{u : x in W_l(u)} U[u] (likewise Vbar):
//   M_U[u] = sum_l L[l]/k^2 sum_{x in W_l(u)} sum_y Vbar_l[y] P[x,y]
//   M_V[v] = sum_l L[l]/k^2 sum_{y in W_l(v)} sum_x Ubar_l[x] P[x,y]
//   M_L[l] = k^-2 sum_{x,y} Ubar_l[x] Vbar_l[y] P[x,y]
//   M_S[s] = sum_{x,y} m_s[x,y][s] gt[x,y] W[x,y],  W = sum_l L[l]/k^2 Ubar_l[x] Vbar_l[y]
//   M_T[t] = sum_{x,y} m_t[x,y][t] gs[x,y] W[x,y]
// (elementwise in the rank r).  One [texels][R] FP64 array holds P during the
// u, v, l updates and W during the s, t updates; gs and gt are recomputed
// where they are needed from factor tiles in LDS.  All FP64.
// ===========================================================================

constexpr int kMassPad = 16;        // largest unrolled bin window
constexpr int kTexThreads = 1024;    // one block shares its LDS factor tiles among 16 wavefronts
constexpr int kMaxLevels = 16;

template <int R>
struct TexTile {
  static constexpr int RT = R < 64 ? R : 64;             // ranks per block (lanes per texel)
  static constexpr int TPW = 64 / RT;                    // texels per wavefront step
  static constexpr int WAVES = kTexThreads / 64;
};

// rows [0, N) x ranks [r0, r0 + RT) of a [N][R] factor into LDS [N][RT]
template <int R>
__device__ __forceinline__ void stage_rank_tile(const double* __restrict__ F, int N, int r0, double* tile) {
  constexpr int RT = TexTile<R>::RT;
  for (int i = threadIdx.x; i < N * RT; i += blockDim.x) tile[i] = F[(i / RT) * R + r0 + i % RT];
}

// sum_j m[j] F[i0 + j][r] over a texel's bin window of P = 2K + 1 bins.  The
// window masses of bins outside [0, N) are zero, so the row is clamped rather
// than tested.  With PMAX > 0 (P <= PMAX) the loop is unrolled to PMAX with
// all loads issued first; the mass array is padded so that reading PMAX
// entries stays inside it, and entries past P are discarded by a select.
template <int RT, int PMAX>
__device__ __forceinline__ double window_dot(const double* __restrict__ m, int i0, int P, int N,
                                             const double* tile, int rr) {
  double acc = 0.0;
  if constexpr (PMAX > 0) {
    double mv[PMAX], tv[PMAX];
#pragma unroll
    for (int j = 0; j < PMAX; ++j) {
      mv[j] = m[j];
      tv[j] = tile[glint_clampi(i0 + j, 0, N - 1) * RT + rr];
    }
#pragma unroll
    for (int j = 0; j < PMAX; ++j) acc += (j < P ? mv[j] : 0.0) * tv[j];
  } else {
    for (int j = 0; j < P; ++j) acc += m[j] * tile[glint_clampi(i0 + j, 0, N - 1) * RT + rr];
  }
  return acc;
}

// The texels [w0, w1) one wavefront walks: a contiguous share of the block's
// chunk, so that runs of texels with one normal (equal bins and window masses)
// stay together.  With 64 or more ranks each step is one texel, the same for
// the whole wavefront.
struct WaveRange {
  int64_t w0, w1;
};
template <int R>
__device__ __forceinline__ WaveRange wave_range(int64_t ntex, int64_t chunk) {
  constexpr int TPW = TexTile<R>::TPW, WAVES = TexTile<R>::WAVES;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t t0 = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t t1 = t0 + chunk < ntex ? t0 + chunk : ntex;
  const int64_t per = ((chunk + WAVES - 1) / WAVES + TPW - 1) / TPW * TPW;
  const int64_t w0 = t0 + wave * per;
  return {w0 < t1 ? w0 : t1, w0 + per < t1 ? w0 + per : t1};
}

__device__ __forceinline__ bool same_normal(float2 a, float2 b) { return a.x == b.x && a.y == b.y; }

// lane k's value of a wavefront-wide register
__device__ __forceinline__ float lane_f(float v, int k) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k));
}

// Pm[tex][r] = gs[tex][r] * gt[tex][r]
template <int R, int PMAX>
__global__ __launch_bounds__(kTexThreads) void k_texel_p(const float2* __restrict__ nxy,
                                                         const int32_t* __restrict__ bins,
                                                         const double* __restrict__ mass, int64_t ntex,
                                                         int K, int N, int64_t chunk,
                                                         const double* __restrict__ S,
                                                         const double* __restrict__ Tf,
                                                         double* __restrict__ Pm, const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  constexpr int RT = TexTile<R>::RT, TPW = TexTile<R>::TPW;
  extern __shared__ __align__(16) double tex_lds[];
  double* sS = tex_lds;
  double* sT = tex_lds + N * RT;
  const int r0 = blockIdx.x * RT;
  stage_rank_tile<R>(S, N, r0, sS);
  stage_rank_tile<R>(Tf, N, r0, sT);
  __syncthreads();
  const int lane = threadIdx.x & 63, rr = lane % RT, tsub = lane / RT;
  const int P = 2 * K + 1;
  const WaveRange wr = wave_range<R>(ntex, chunk);
  const int2* b2 = reinterpret_cast<const int2*>(bins);
  float2 prev = make_float2(__builtin_nanf(""), 0.0f);
  double val = 0.0;
  if constexpr (TPW == 1) {
    // one texel per step for the whole wavefront: the normals and bins of 64
    // texels come in one vector load and are read out lane by lane
    for (int64_t tb = wr.w0; tb < wr.w1; tb += 64) {
      const int nb = static_cast<int>(wr.w1 - tb < 64 ? wr.w1 - tb : 64);
      const float2 nm = lane < nb ? nxy[tb + lane] : make_float2(0.0f, 0.0f);
      const int2 bm = lane < nb ? b2[tb + lane] : make_int2(0, 0);
      for (int k = 0; k < nb; ++k) {
        const float2 n = make_float2(lane_f(nm.x, k), lane_f(nm.y, k));
        const int64_t tex = tb + k;
        if (!same_normal(n, prev)) {
          const int bx = __builtin_amdgcn_readlane(bm.x, k), by = __builtin_amdgcn_readlane(bm.y, k);
          const double* ms = mass + tex * 2 * P;
          val = window_dot<RT, PMAX>(ms, bx - K, P, N, sS, rr) * window_dot<RT, PMAX>(ms + P, by - K, P, N, sT, rr);
          prev = n;
        }
        Pm[tex * R + r0 + rr] = val;
      }
    }
  } else {
    for (int64_t tb = wr.w0; tb < wr.w1; tb += TPW) {
      const int64_t tex = tb + tsub;
      if (tex < wr.w1) {
        const float2 n = nxy[tex];
        if (!same_normal(n, prev)) {
          const int2 b = b2[tex];
          const double* ms = mass + tex * 2 * P;
          val = window_dot<RT, PMAX>(ms, b.x - K, P, N, sS, rr) *
                window_dot<RT, PMAX>(ms + P, b.y - K, P, N, sT, rr);
          prev = n;
        }
        Pm[tex * R + r0 + rr] = val;
      }
    }
  }
}

// Window contraction over the inner texel axis, XT outer rows per thread and
// the inner axis split over gridDim.y:
//   ROWS:  H[l][x][r] = sum_y Wb[l][y][r] Pm[x][y][r]      (outer x, inner y)
//   !ROWS: H[l][y][r] = sum_x Wb[l][x][r] Pm[x][y][r]      (outer y, inner x)
//   ML (with ROWS): M[l][r] += k^-2 sum_x Ub[l][x][r] H[l][x][r] in place of H.
// NL is the level count rounded up to a multiple of 4; the window sums are
// zero on the padding levels, which are not stored.  The P and window-sum
// values of the next inner step are loaded while the current one is used.
// The destination must be zero on entry when gridDim.y > 1 or ML.
template <int R, int XT, int NL, bool ROWS, bool ML>
__global__ __launch_bounds__(256) void k_texel_contract(const double* __restrict__ Pm,
                                                        const double* __restrict__ Wb,
                                                        const double* __restrict__ Ub, int nu, int nv,
                                                        int nl, int ichunk, double* __restrict__ H,
                                                        const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  const int outer = ROWS ? nu : nv, inner = ROWS ? nv : nu;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = static_cast<int>(idx % R);
  const int o0 = static_cast<int>(idx / R) * XT;
  if (o0 >= outer) return;
  const int i0 = blockIdx.y * ichunk;
  const int i1 = min(i0 + ichunk, inner);
  if (i0 >= i1) return;
  // P[o][i] at pp[o] + i * istep
  const double* pp[XT];
#pragma unroll
  for (int xt = 0; xt < XT; ++xt) {
    const int o = min(o0 + xt, outer - 1);
    pp[xt] = Pm + (ROWS ? static_cast<int64_t>(o) * nv : o) * R + r;
  }
  const int64_t istep = ROWS ? R : static_cast<int64_t>(nv) * R;
  const double* wp = Wb + r;
  const int64_t lstride = static_cast<int64_t>(inner) * R;
  double acc[XT][NL];
#pragma unroll
  for (int xt = 0; xt < XT; ++xt)
#pragma unroll
    for (int l = 0; l < NL; ++l) acc[xt][l] = 0.0;
  double pn[XT], wn[NL];
#pragma unroll
  for (int xt = 0; xt < XT; ++xt) pn[xt] = pp[xt][i0 * istep];
#pragma unroll
  for (int l = 0; l < NL; ++l) wn[l] = wp[l * lstride + static_cast<int64_t>(i0) * R];
  for (int i = i0; i < i1; ++i) {
    double p[XT], w[NL];
#pragma unroll
    for (int xt = 0; xt < XT; ++xt) p[xt] = pn[xt];
#pragma unroll
    for (int l = 0; l < NL; ++l) w[l] = wn[l];
    const int in = i + 1 < i1 ? i + 1 : i;
#pragma unroll
    for (int xt = 0; xt < XT; ++xt) pn[xt] = pp[xt][in * istep];
#pragma unroll
    for (int l = 0; l < NL; ++l) wn[l] = wp[l * lstride + static_cast<int64_t>(in) * R];
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
      for (int xt = 0; xt < XT; ++xt) acc[xt][l] += w[l] * p[xt];
  }
  if constexpr (ML) {
#pragma unroll
    for (int l = 0; l < NL; ++l)
      if (l < nl) {
        double sum = 0.0;
#pragma unroll
        for (int xt = 0; xt < XT; ++xt)
          if (o0 + xt < outer) sum += acc[xt][l] * Ub[(static_cast<int64_t>(l) * nu + o0 + xt) * R + r];
        const double k = static_cast<double>(1 << l);
        atomicAdd(&H[l * R + r], sum / (k * k));
      }
  } else {
#pragma unroll
    for (int xt = 0; xt < XT; ++xt)
      if (o0 + xt < outer)
#pragma unroll
        for (int l = 0; l < NL; ++l)
          if (l < nl) {
            double* dst = &H[(static_cast<int64_t>(l) * outer + o0 + xt) * R + r];
            if (gridDim.y > 1) atomicAdd(dst, acc[xt][l]);
            else *dst = acc[xt][l];
          }
  }
}

// Wt[x][y][r] = sum_l L[l][r] / k^2 Ub[l][x][r] Vb[l][y][r], XT rows x per
// thread, y split over gridDim.y.  Up to 8 levels the next y's window sums
// are loaded ahead; at 12 levels the loads-ahead would take the kernel past
// 256 VGPRs, one wavefront a SIMD, and without them it runs two (measured at
// 4096^2 texels, rank 256: 14.8 -> 11.4 ms; 2048^2, rank 128, 10 levels:
// 1.72 -> 1.36 ms)
template <int R, int XT, int NL>
__global__ __launch_bounds__(256) void k_texel_w(const double* __restrict__ Ub, const double* __restrict__ Vb,
                                                 const double* __restrict__ L, int nu, int nv, int nl,
                                                 int ychunk, double* __restrict__ Wt,
                                                 const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = static_cast<int>(idx % R);
  const int x0 = static_cast<int>(idx / R) * XT;
  if (x0 >= nu) return;
  const int y0 = blockIdx.y * ychunk;
  const int y1 = min(y0 + ychunk, nv);
  if (y0 >= y1) return;
  double a[XT][NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    const double k = static_cast<double>(1 << l);
    const double c = l < nl ? L[l * R + r] / (k * k) : 0.0;
#pragma unroll
    for (int xt = 0; xt < XT; ++xt)
      a[xt][l] = c * Ub[(static_cast<int64_t>(l) * nu + min(x0 + xt, nu - 1)) * R + r];
  }
  const int64_t lstride = static_cast<int64_t>(nv) * R;
  const double* vp = Vb + r;
  double* wp[XT];
#pragma unroll
  for (int xt = 0; xt < XT; ++xt) wp[xt] = Wt + static_cast<int64_t>(min(x0 + xt, nu - 1)) * nv * R + r;
  constexpr bool kAhead = NL <= 8;
  double vn[NL];
  if constexpr (kAhead) {
#pragma unroll
    for (int l = 0; l < NL; ++l) vn[l] = vp[l * lstride + static_cast<int64_t>(y0) * R];
  }
  for (int y = y0; y < y1; ++y) {
    double v[NL];
    if constexpr (kAhead) {
#pragma unroll
      for (int l = 0; l < NL; ++l) v[l] = vn[l];
      const int yn = y + 1 < y1 ? y + 1 : y;
#pragma unroll
      for (int l = 0; l < NL; ++l) vn[l] = vp[l * lstride + static_cast<int64_t>(yn) * R];
    } else {
#pragma unroll
      for (int l = 0; l < NL; ++l) v[l] = vp[l * lstride + static_cast<int64_t>(y) * R];
    }
    double w[XT];
#pragma unroll
    for (int xt = 0; xt < XT; ++xt) w[xt] = 0.0;
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
      for (int xt = 0; xt < XT; ++xt) w[xt] += a[xt][l] * v[l];
#pragma unroll
    for (int xt = 0; xt < XT; ++xt)
      if (x0 + xt < nu) wp[xt][static_cast<int64_t>(y) * R] = w[xt];
  }
}

// Mode s (AXIS 0) or t (AXIS 1): every texel adds its AXIS bin-window masses
// times q = g * Wt[tex][r] to the rows of its window, g being the contraction
// of the other axis' window with that axis' factor F.  A run of texels with
// one normal shares g and the masses, so it adds g * (sum of its Wt) once.  A
// block sums a chunk of texels for RT ranks in LDS and stores the tile in its
// slot of parts[chunk][N][R]; the slots are summed afterwards (fixed order).
template <int R, int AXIS, int PMAX>
__global__ __launch_bounds__(kTexThreads) void k_texel_scatter(const float2* __restrict__ nxy,
                                                               const int32_t* __restrict__ bins,
                                                               const double* __restrict__ mass, int64_t ntex,
                                                               int K, int N, int64_t chunk,
                                                               const double* __restrict__ F,
                                                               const double* __restrict__ Wt,
                                                               double* __restrict__ parts,
                                                               const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  constexpr int RT = TexTile<R>::RT, TPW = TexTile<R>::TPW;
  extern __shared__ __align__(16) double tex_lds[];
  double* acc = tex_lds;             // [N][RT]
  double* sF = tex_lds + N * RT;     // [N][RT]
  const int r0 = blockIdx.x * RT;
  for (int i = threadIdx.x; i < N * RT; i += blockDim.x) acc[i] = 0.0;
  stage_rank_tile<R>(F, N, r0, sF);
  __syncthreads();
  const int lane = threadIdx.x & 63, rr = lane % RT, tsub = lane / RT;
  const int P = 2 * K + 1;
  const WaveRange wr = wave_range<R>(ntex, chunk);
  const int2* b2 = reinterpret_cast<const int2*>(bins);
  float2 prev = make_float2(__builtin_nanf(""), 0.0f);
  const double* mo = nullptr;
  int i0 = 0;
  double g = 0.0, wsum = 0.0;
  auto flush = [&]() {
    if (mo == nullptr) return;
    const double q = g * wsum;
    if constexpr (PMAX > 0) {
      double mv[PMAX];
#pragma unroll
      for (int j = 0; j < PMAX; ++j) mv[j] = mo[j];
#pragma unroll
      for (int j = 0; j < PMAX; ++j) {
        const int i = i0 + j;
        if (j < P && i >= 0 && i < N) atomicAdd(&acc[i * RT + rr], mv[j] * q);
      }
    } else {
      for (int j = 0; j < P; ++j) {
        const int i = i0 + j;
        if (i >= 0 && i < N) atomicAdd(&acc[i * RT + rr], mo[j] * q);
      }
    }
  };
  auto start_run = [&](int64_t tex, float2 n, int bx, int by) {
    flush();
    mo = mass + (2 * tex + AXIS) * P;
    i0 = (AXIS ? by : bx) - K;
    g = window_dot<RT, PMAX>(mass + (2 * tex + (1 - AXIS)) * P, (AXIS ? bx : by) - K, P, N, sF, rr);
    wsum = 0.0;
    prev = n;
  };
  if constexpr (TPW == 1) {
    // one texel per step for the whole wavefront; normals and bins of 64
    // texels per vector load, the Wt rows of the next 8 texels in flight
    constexpr int kG = 8;
    const double* wrow = Wt + r0 + rr;
    for (int64_t tb = wr.w0; tb < wr.w1; tb += 64) {
      const int nb = static_cast<int>(wr.w1 - tb < 64 ? wr.w1 - tb : 64);
      const float2 nm = lane < nb ? nxy[tb + lane] : make_float2(0.0f, 0.0f);
      const int2 bm = lane < nb ? b2[tb + lane] : make_int2(0, 0);
      double wa[kG], wb[kG];
#pragma unroll
      for (int j = 0; j < kG; ++j) wa[j] = wrow[(tb + min(j, nb - 1)) * R];
      for (int k0 = 0; k0 < nb; k0 += kG) {
#pragma unroll
        for (int j = 0; j < kG; ++j) wb[j] = wrow[(tb + min(k0 + kG + j, nb - 1)) * R];
#pragma unroll
        for (int j = 0; j < kG; ++j) {
          const int k = k0 + j;
          if (k < nb) {
            const float2 n = make_float2(lane_f(nm.x, k), lane_f(nm.y, k));
            if (!same_normal(n, prev))
              start_run(tb + k, n, __builtin_amdgcn_readlane(bm.x, k), __builtin_amdgcn_readlane(bm.y, k));
            wsum += wa[j];
          }
        }
#pragma unroll
        for (int j = 0; j < kG; ++j) wa[j] = wb[j];
      }
    }
  } else {
    for (int64_t tb = wr.w0; tb < wr.w1; tb += TPW) {
      const int64_t tex = tb + tsub;
      if (tex < wr.w1) {
        const float2 n = nxy[tex];
        if (!same_normal(n, prev)) {
          const int2 b = b2[tex];
          start_run(tex, n, b.x, b.y);
        }
        wsum += Wt[tex * R + r0 + rr];
      }
    }
  }
  flush();
  __syncthreads();
  double* dst = parts + static_cast<int64_t>(blockIdx.y) * N * R;
  for (int i = threadIdx.x; i < N * RT; i += blockDim.x) dst[(i / RT) * R + r0 + i % RT] = acc[i];
}

// C[g][j][r] = sum_{i<j} X[g][i][r], j = 0..n, for `groups` stacked [n][R]
// blocks: one block per (group, tile of up to 64 ranks), the rows cut into
// segments summed in parallel.
__global__ __launch_bounds__(1024) void k_prefix_rows(const double* __restrict__ X, int n, int R,
                                                      double* __restrict__ C, const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  __shared__ double seg[1024];
  const int RB = R < 64 ? R : 64;
  const int parts = blockDim.x / RB;
  const int rr = threadIdx.x % RB, part = threadIdx.x / RB;
  const int r = blockIdx.x * RB + rr;
  const double* x = X + static_cast<int64_t>(blockIdx.y) * n * R + r;
  double* c = C + static_cast<int64_t>(blockIdx.y) * (n + 1) * R + r;
  const int len = (n + parts - 1) / parts;
  const int a = min(part * len, n), e = min(a + len, n);
  double s = 0.0;
  for (int i = a; i < e; ++i) s += x[static_cast<int64_t>(i) * R];
  seg[threadIdx.x] = s;
  __syncthreads();
  double off = 0.0;
  for (int p = 0; p < part; ++p) off += seg[p * RB + rr];
  if (part == 0) c[0] = 0.0;
  for (int i = a; i < e; ++i) {
    off += x[static_cast<int64_t>(i) * R];
    c[static_cast<int64_t>(i + 1) * R] = off;
  }
}

// Sum of X[m mod n] over the integer range [lo, hi), from its prefix table C
// (C[j] = sum_{i<j} X[i], j = 0..n).
__device__ __forceinline__ double wrap_range_sum(const double* C, int n, int R, int lo, int hi) {
  auto pf = [&](int m) {
    const int w = m >= 0 ? m / n : -((-m + n - 1) / n);
    const int rr = m - w * n;
    return static_cast<double>(w) * C[static_cast<int64_t>(n) * R] + C[static_cast<int64_t>(rr) * R];
  };
  return pf(hi) - pf(lo);
}

// out[l][x][r] = sum of F[c][r] over the centres c whose level-l footprint covers x,
// i.e. c in [x + h - k + 1, x + h] (k = 2^l, h = k/2), wrapping.
__global__ void k_window_sums(const double* __restrict__ Cpref, int n, int R, int nl,
                              double* __restrict__ out, const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  const int64_t total = static_cast<int64_t>(nl) * n * R;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int r = static_cast<int>(idx % R);
    const int64_t t = idx / R;
    const int x = static_cast<int>(t % n), l = static_cast<int>(t / n);
    const int k = 1 << l, h = k >> 1;
    out[idx] = wrap_range_sum(Cpref + r, n, R, x + h - k + 1, x + h + 1);
  }
}

// M[c][r] = sum_l L[l][r]/k^2 * sum_{x in W_l(c)} H[l][x][r], W_l(c) = [c - h, c - h + k).
__global__ void k_window_apply(const double* __restrict__ Hpref, int n, int R, int nl,
                               const double* __restrict__ L, double* __restrict__ M,
                               const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * R) return;
  const int c = idx / R, r = idx % R;
  double acc = 0.0;
  for (int l = 0; l < nl; ++l) {
    const int k = 1 << l, h = k >> 1;
    const double s = wrap_range_sum(Hpref + static_cast<int64_t>(l) * (n + 1) * R + r, n, R, c - h, c - h + k);
    acc += L[l * R + r] / (static_cast<double>(k) * k) * s;
  }
  M[idx] = acc;
}

// G = A^T A over a chunk of rows per blockIdx.z, into parts[z][R][R]: 16 x 16
// output tiles, rows staged through LDS.
__global__ __launch_bounds__(256) void k_gram_parts(const double* __restrict__ A, int rows, int R, int rchunk,
                                                    double* __restrict__ parts, const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  __shared__ double ai[32][17], aj[32][17];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
  const int k0 = blockIdx.z * rchunk, k1 = min(k0 + rchunk, rows);
  double acc = 0.0;
  for (int kb = k0; kb < k1; kb += 32) {
    for (int e = threadIdx.x; e < 32 * 16; e += 256) {
      const int kk = e / 16, c = e % 16;
      const bool in = kb + kk < k1;
      ai[kk][c] = in ? A[static_cast<int64_t>(kb + kk) * R + blockIdx.y * 16 + c] : 0.0;
      aj[kk][c] = in ? A[static_cast<int64_t>(kb + kk) * R + blockIdx.x * 16 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < 32; ++kk) acc += ai[kk][ty] * aj[kk][tx];
    __syncthreads();
  }
  parts[static_cast<int64_t>(blockIdx.z) * R * R + i * R + j] = acc;
}

// Fixed-order sum of the per-chunk partial tiles parts[p][n] in two levels:
// each group of kPartGroup consecutive tiles is summed into its first tile,
// then the group heads into out.
constexpr int kPartGroup = 32;
__global__ void k_sum_part_groups(double* __restrict__ parts, int nparts, int64_t n, const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p0 = blockIdx.y * kPartGroup;
  const int p1 = min(p0 + kPartGroup, nparts);
  double acc = 0.0;
  for (int p = p0; p < p1; ++p) acc += parts[p * n + i];
  parts[p0 * n + i] = acc;
}

__global__ void k_sum_group_heads(const double* __restrict__ parts, int groups, int64_t n, double* __restrict__ out,
                                  const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int g = 0; g < groups; ++g) acc += parts[static_cast<int64_t>(g) * kPartGroup * n + i];
  out[i] = acc;
}

struct TexelLayout {
  size_t bins, mass, pm, ub, vb, hb, hpref, cpre, parts, gparts, m, grams, lc, lct, lam, scal, ctrl, total;
  int64_t chunk_p, chunk_s, nchunk_s;
  int gsplit;
};

constexpr int kGramRowsPerSplit = 256;

void texel_layout(const glint_ndf_desc* d, int R, TexelLayout* L) {
  const int64_t ntex = static_cast<int64_t>(d->nu) * d->nv;
  const int K = glint_window_k(d);
  const size_t P = 2 * K + 1;
  const size_t nmax = std::max(d->nu, d->nv);
  const size_t rows = std::max<size_t>(nmax, std::max(d->nlevels, d->nbins));
  const int RT = R < 64 ? R : 64;
  // chunks of the texel kernels: >= 4096 texels per block for the P pass, about
  // 2048 blocks for the scatter passes (whose per-chunk tiles are summed later)
  L->chunk_p = std::max<int64_t>(4096, (ntex + 65534) / 65535);
  const int64_t want = std::max<int64_t>(1, 2048 / (R / RT));
  L->chunk_s = std::max<int64_t>(512, (ntex + want - 1) / want);
  L->nchunk_s = (ntex + L->chunk_s - 1) / L->chunk_s;
  L->gsplit = static_cast<int>((rows + kGramRowsPerSplit - 1) / kGramRowsPerSplit);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += glint_round_up(bytes, 256);
    return at;
  };
  L->bins = take(sizeof(int32_t) * 2 * ntex);
  L->mass = take(sizeof(double) * (2 * ntex * P + kMassPad));   // padded for the unrolled window reads
  L->pm = take(sizeof(double) * ntex * R);
  const int nlp = (d->nlevels + 3) / 4 * 4;   // levels padded to a multiple of 4
  L->ub = take(sizeof(double) * nlp * d->nu * R);
  L->vb = take(sizeof(double) * nlp * d->nv * R);
  L->hb = take(sizeof(double) * d->nlevels * nmax * R);
  L->hpref = take(sizeof(double) * d->nlevels * (nmax + 1) * R);
  L->cpre = take(sizeof(double) * (nmax + 1) * R);
  L->parts = take(sizeof(double) * L->nchunk_s * d->nbins * R);
  L->gparts = take(sizeof(double) * L->gsplit * R * R);
  L->m = take(sizeof(double) * rows * R);
  L->grams = take(sizeof(double) * 5 * R * R);
  L->lc = take(sizeof(double) * R * R);
  L->lct = take(sizeof(double) * R * R);
  L->lam = take(sizeof(double) * R);
  L->scal = take(sizeof(double) * 4);
  L->ctrl = take(sizeof(int) * CTRL_N);
  L->total = off;
}

struct TexelCtx {
  const glint_ndf_desc* d;
  const float2* nxy;
  int R;
  const TexelLayout* lo;
  int K;
  int32_t* bins;
  double *mass, *pm, *ub, *vb, *hb, *hpref, *cpre, *parts, *gparts, *M;
  int* ctrl;
  hipStream_t stream;
};

// the window-sum levels beyond nlevels (padding to a multiple of 4) are read
// as zeros by the contraction kernels
void texel_zero_padding(const TexelCtx& c) {
  const int nl = c.d->nlevels, nlp = (nl + 3) / 4 * 4;
  if (nlp == nl) return;
  const int R = c.R;
  const int64_t nu_pad = static_cast<int64_t>(nlp - nl) * c.d->nu * R;
  const int64_t nv_pad = static_cast<int64_t>(nlp - nl) * c.d->nv * R;
  hipLaunchKernelGGL(k_zero, dim3(static_cast<unsigned>(std::min<int64_t>((nu_pad + 255) / 256, 4096))), dim3(256),
                     0, c.stream, c.ub + static_cast<int64_t>(nl) * c.d->nu * R, nu_pad, c.ctrl);
  hipLaunchKernelGGL(k_zero, dim3(static_cast<unsigned>(std::min<int64_t>((nv_pad + 255) / 256, 4096))), dim3(256),
                     0, c.stream, c.vb + static_cast<int64_t>(nl) * c.d->nv * R, nv_pad, c.ctrl);
}

void texel_ctx(const glint_ndf_desc* d, const float* nxy, const TexelLayout& Lo, unsigned char* ws, double* M,
               hipStream_t stream, TexelCtx* c) {
  c->d = d;
  c->nxy = reinterpret_cast<const float2*>(nxy);
  c->R = 0;
  c->lo = &Lo;
  c->K = glint_window_k(d);
  c->stream = stream;
  c->bins = reinterpret_cast<int32_t*>(ws + Lo.bins);
  c->mass = reinterpret_cast<double*>(ws + Lo.mass);
  c->pm = reinterpret_cast<double*>(ws + Lo.pm);
  c->ub = reinterpret_cast<double*>(ws + Lo.ub);
  c->vb = reinterpret_cast<double*>(ws + Lo.vb);
  c->hb = reinterpret_cast<double*>(ws + Lo.hb);
  c->hpref = reinterpret_cast<double*>(ws + Lo.hpref);
  c->cpre = reinterpret_cast<double*>(ws + Lo.cpre);
  c->parts = reinterpret_cast<double*>(ws + Lo.parts);
  c->gparts = reinterpret_cast<double*>(ws + Lo.gparts);
  c->M = M ? M : reinterpret_cast<double*>(ws + Lo.m);
  c->ctrl = reinterpret_cast<int*>(ws + Lo.ctrl);
}

// outer rows per thread and inner split of the contraction kernels: about
// 2^17 threads, at least 32 inner steps per thread
constexpr int kTexXT = 8;
inline int inner_split(int outer, int inner, int R) {
  const int64_t threads = static_cast<int64_t>((outer + kTexXT - 1) / kTexXT) * R;
  int64_t s = ((int64_t{1} << 17) + threads - 1) / threads;
  s = std::min<int64_t>(s, std::max(1, inner / 32));
  return static_cast<int>(std::max<int64_t>(s, 1));
}

// the unrolled bin-window bound for a window of P bins (0: not unrolled)
inline int window_pmax(int P) { return P <= 8 ? 8 : (P <= kMassPad ? kMassPad : 0); }

template <int R, int PMAX>
void texel_p_pm(const TexelCtx& c, const double* S, const double* Tf) {
  constexpr int RT = TexTile<R>::RT;
  const int64_t ntex = static_cast<int64_t>(c.d->nu) * c.d->nv;
  const dim3 grid(R / RT, static_cast<unsigned>((ntex + c.lo->chunk_p - 1) / c.lo->chunk_p));
  hipLaunchKernelGGL((k_texel_p<R, PMAX>), grid, dim3(kTexThreads), sizeof(double) * 2 * c.d->nbins * RT,
                     c.stream, c.nxy, c.bins, c.mass, ntex, c.K, c.d->nbins, c.lo->chunk_p, S, Tf, c.pm, c.ctrl);
}

template <int R>
void texel_p(const TexelCtx& c, const double* S, const double* Tf) {
  switch (window_pmax(2 * c.K + 1)) {
    case 8: texel_p_pm<R, 8>(c, S, Tf); break;
    case kMassPad: texel_p_pm<R, kMassPad>(c, S, Tf); break;
    default: texel_p_pm<R, 0>(c, S, Tf); break;
  }
}

template <int R, int AXIS, int PMAX>
void texel_scatter_pm(const TexelCtx& c, const double* F, dim3 grid, size_t lds) {
  const int64_t ntex = static_cast<int64_t>(c.d->nu) * c.d->nv;
  hipLaunchKernelGGL((k_texel_scatter<R, AXIS, PMAX>), grid, dim3(kTexThreads), lds, c.stream, c.nxy, c.bins,
                     c.mass, ntex, c.K, c.d->nbins, c.lo->chunk_s, F, c.pm, c.parts, c.ctrl);
}

template <int R, int AXIS>
void texel_scatter(const TexelCtx& c, const double* F, dim3 grid, size_t lds) {
  switch (window_pmax(2 * c.K + 1)) {
    case 8: texel_scatter_pm<R, AXIS, 8>(c, F, grid, lds); break;
    case kMassPad: texel_scatter_pm<R, AXIS, kMassPad>(c, F, grid, lds); break;
    default: texel_scatter_pm<R, AXIS, 0>(c, F, grid, lds); break;
  }
}

template <int R>
void texel_window(const TexelCtx& c, const double* F, int n, double* out) {
  const int nl = c.d->nlevels;
  const int RB = R < 64 ? R : 64;
  hipLaunchKernelGGL(k_prefix_rows, dim3(R / RB, 1), dim3(1024), 0, c.stream, F, n, R, c.cpre, c.ctrl);
  const int64_t total = static_cast<int64_t>(nl) * n * R;
  hipLaunchKernelGGL(k_window_sums, dim3(static_cast<unsigned>(std::min<int64_t>((total + 255) / 256, 1 << 16))),
                     dim3(256), 0, c.stream, c.cpre, n, R, nl, out, c.ctrl);
}

template <int R, int NL>
void texel_w_nl(const TexelCtx& c, const double* L, dim3 grid, int ychunk) {
  hipLaunchKernelGGL((k_texel_w<R, kTexXT, NL>), grid, dim3(256), 0, c.stream, c.ub, c.vb, L, c.d->nu, c.d->nv,
                     c.d->nlevels, ychunk, c.pm, c.ctrl);
}

template <int R>
void texel_w(const TexelCtx& c, const double* L) {
  const int nu = c.d->nu, nv = c.d->nv;
  const int split = inner_split(nu, nv, R);
  const int ychunk = (nv + split - 1) / split;
  const int64_t threads = static_cast<int64_t>((nu + kTexXT - 1) / kTexXT) * R;
  const dim3 grid(static_cast<unsigned>((threads + 255) / 256), static_cast<unsigned>((nv + ychunk - 1) / ychunk));
  switch ((c.d->nlevels + 3) / 4) {
    case 1: texel_w_nl<R, 4>(c, L, grid, ychunk); break;
    case 2: texel_w_nl<R, 8>(c, L, grid, ychunk); break;
    case 3: texel_w_nl<R, 12>(c, L, grid, ychunk); break;
    default: texel_w_nl<R, 16>(c, L, grid, ychunk); break;
  }
}

template <int R, int NL>
void texel_contract_nl(const TexelCtx& c, int mode, dim3 grid, int ichunk, double* dst) {
  const int nu = c.d->nu, nv = c.d->nv, nl = c.d->nlevels;
  hipStream_t st = c.stream;
  if (mode == 0)
    hipLaunchKernelGGL((k_texel_contract<R, kTexXT, NL, true, false>), grid, dim3(256), 0, st, c.pm, c.vb,
                       static_cast<const double*>(nullptr), nu, nv, nl, ichunk, dst, c.ctrl);
  else if (mode == 1)
    hipLaunchKernelGGL((k_texel_contract<R, kTexXT, NL, false, false>), grid, dim3(256), 0, st, c.pm, c.ub,
                       static_cast<const double*>(nullptr), nu, nv, nl, ichunk, dst, c.ctrl);
  else
    hipLaunchKernelGGL((k_texel_contract<R, kTexXT, NL, true, true>), grid, dim3(256), 0, st, c.pm, c.vb, c.ub,
                       nu, nv, nl, ichunk, dst, c.ctrl);
}

// The contraction of one mode into c.M.  Requires: modes u, v, l: P in c.pm and
// the window sums of the other spatial factor(s) current; modes s, t: W in c.pm.
template <int R>
glint_status texel_mode(const TexelCtx& c, int mode, const double* L, const double* S, const double* Tf) {
  const glint_ndf_desc* d = c.d;
  const int nu = d->nu, nv = d->nv, nl = d->nlevels, N = d->nbins;
  hipStream_t st = c.stream;
  if (mode <= 2) {
    const bool rows = mode != 1;
    const int outer = rows ? nu : nv, inner = rows ? nv : nu;
    const int split = inner_split(outer, inner, R);
    const int ichunk = (inner + split - 1) / split;
    const int64_t threads = static_cast<int64_t>((outer + kTexXT - 1) / kTexXT) * R;
    const dim3 grid(static_cast<unsigned>((threads + 255) / 256),
                    static_cast<unsigned>((inner + ichunk - 1) / ichunk));
    double* dst = mode == 2 ? c.M : c.hb;
    const int64_t n = mode == 2 ? static_cast<int64_t>(nl) * R : static_cast<int64_t>(nl) * outer * R;
    if (mode == 2 || grid.y > 1)
      hipLaunchKernelGGL(k_zero, dim3(static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 4096))), dim3(256),
                         0, st, dst, n, c.ctrl);
    switch ((nl + 3) / 4) {
      case 1: texel_contract_nl<R, 4>(c, mode, grid, ichunk, dst); break;
      case 2: texel_contract_nl<R, 8>(c, mode, grid, ichunk, dst); break;
      case 3: texel_contract_nl<R, 12>(c, mode, grid, ichunk, dst); break;
      default: texel_contract_nl<R, 16>(c, mode, grid, ichunk, dst); break;
    }
    if (mode <= 1) {
      const int RB = R < 64 ? R : 64;
      hipLaunchKernelGGL(k_prefix_rows, dim3(R / RB, nl), dim3(1024), 0, st, c.hb, outer, R, c.hpref, c.ctrl);
      hipLaunchKernelGGL(k_window_apply, dim3((outer * R + 255) / 256), dim3(256), 0, st, c.hpref, outer, R, nl,
                         L, c.M, c.ctrl);
    }
    GLINT_LAUNCHED("texel modes u, v, l");
    return GLINT_OK;
  }
  constexpr int RT = TexTile<R>::RT;
  const int64_t ntex = static_cast<int64_t>(nu) * nv;
  const dim3 grid(R / RT, static_cast<unsigned>(c.lo->nchunk_s));
  const size_t lds = sizeof(double) * 2 * N * RT;
  if (mode == 3) texel_scatter<R, 0>(c, Tf, grid, lds);
  else texel_scatter<R, 1>(c, S, grid, lds);
  const int64_t n = static_cast<int64_t>(N) * R;
  const int nparts = static_cast<int>(c.lo->nchunk_s);
  const int groups = (nparts + kPartGroup - 1) / kPartGroup;
  hipLaunchKernelGGL(k_sum_part_groups, dim3(static_cast<unsigned>((n + 255) / 256), groups), dim3(256), 0, st,
                     c.parts, nparts, n, c.ctrl);
  hipLaunchKernelGGL(k_sum_group_heads, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, c.parts,
                     groups, n, c.M, c.ctrl);
  GLINT_LAUNCHED("texel modes s, t");
  return GLINT_OK;
}

// G = sum of the row-chunk partial Grams
__global__ void k_gram_reduce(const double* __restrict__ parts, int nsplit, int64_t n, double* __restrict__ G,
                              const int* __restrict__ ctrl) {
  if (ctrl[CTRL_DONE]) return;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double acc = 0.0;
    for (int p = 0; p < nsplit; ++p) acc += parts[p * n + i];
    G[i] = acc;
  }
}

template <int R>
void texel_gram(const TexelCtx& c, const double* A, int rows, double* G) {
  const int split = (rows + kGramRowsPerSplit - 1) / kGramRowsPerSplit;
  hipLaunchKernelGGL(k_gram_parts, dim3(R / 16, R / 16, split), dim3(256), 0, c.stream, A, rows, R,
                     kGramRowsPerSplit, c.gparts, c.ctrl);
  const int64_t n = static_cast<int64_t>(R) * R;
  hipLaunchKernelGGL(k_gram_reduce, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, c.stream,
                     c.gparts, split, n, G, c.ctrl);
}

template <int R>
glint_status run_texel_als(const glint_ndf_desc* d, const float* nxy, int iters, double tol, double normT2,
                           double* F[5], double* fit_hist, int32_t* info, unsigned char* ws,
                           const TexelLayout& Lo, hipStream_t stream) {
  const int nu = d->nu, nv = d->nv, nl = d->nlevels, N = d->nbins;
  const int rows[5] = {nu, nv, nl, N, N};
  TexelCtx c;
  texel_ctx(d, nxy, Lo, ws, nullptr, stream, &c);
  double* grams = reinterpret_cast<double*>(ws + Lo.grams);
  double* Lc = reinterpret_cast<double*>(ws + Lo.lc);
  double* LcT = reinterpret_cast<double*>(ws + Lo.lct);
  double* lam = reinterpret_cast<double*>(ws + Lo.lam);
  double* scal = reinterpret_cast<double*>(ws + Lo.scal);
  glint_status st = glint_texel_bins(d, nxy, c.bins, c.mass, stream);
  if (st != GLINT_OK) return st;
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_als_init, dim3(1), dim3(64), 0, stream, c.ctrl, scal + 1, lam, R);
  hipLaunchKernelGGL(k_fill_scalar, dim3(1), dim3(1), 0, stream, scal, normT2);
  c.R = R;
  texel_zero_padding(c);
  for (int m = 0; m < 5; ++m) texel_gram<R>(c, F[m], rows[m], grams + m * R * R);
  GLINT_LAUNCHED("texel ALS init");
  auto update = [&](int n) -> glint_status {
    hipLaunchKernelGGL((k_cholesky<R>), dim3(1), dim3(cholesky_grid(R) * cholesky_grid(R)), 0, stream, grams, n, Lc,
                       LcT, c.ctrl);
    hipLaunchKernelGGL((k_eigh_pinv<R>), dim3(1), dim3(1024), 0, stream, grams, n, Lc, LcT, c.ctrl);
    hipLaunchKernelGGL((k_solve<R>), dim3((rows[n] + 15) / 16), dim3(1024), solve_lds_bytes<R>(), stream, c.M,
                       rows[n], Lc, LcT,
                       F[n], c.ctrl);
    hipLaunchKernelGGL(k_normalize_gram, dim3(1), dim3(1024), 0, stream, F[n], rows[n], R, lam,
                       static_cast<double*>(nullptr), c.ctrl);
    texel_gram<R>(c, F[n], rows[n], grams + n * R * R);
    GLINT_LAUNCHED("texel ALS update");
    return GLINT_OK;
  };
  for (int it = 0; it < iters; ++it) {
    texel_p<R>(c, F[3], F[4]);
    texel_window<R>(c, F[1], nv, c.vb);
    if ((st = texel_mode<R>(c, 0, F[2], F[3], F[4])) != GLINT_OK || (st = update(0)) != GLINT_OK) return st;
    texel_window<R>(c, F[0], nu, c.ub);
    if ((st = texel_mode<R>(c, 1, F[2], F[3], F[4])) != GLINT_OK || (st = update(1)) != GLINT_OK) return st;
    texel_window<R>(c, F[1], nv, c.vb);
    if ((st = texel_mode<R>(c, 2, F[2], F[3], F[4])) != GLINT_OK || (st = update(2)) != GLINT_OK) return st;
    texel_w<R>(c, F[2]);
    if ((st = texel_mode<R>(c, 3, F[2], F[3], F[4])) != GLINT_OK || (st = update(3)) != GLINT_OK) return st;
    if ((st = texel_mode<R>(c, 4, F[2], F[3], F[4])) != GLINT_OK || (st = update(4)) != GLINT_OK) return st;
    hipLaunchKernelGGL(k_fit, dim3(1), dim3(256), 0, stream, grams, lam, c.M, F[4], N, R, scal, it, tol, fit_hist,
                       scal + 1, c.ctrl);
    GLINT_LAUNCHED("k_fit");
  }
  hipLaunchKernelGGL(k_absorb, dim3((nl * R + 255) / 256), dim3(256), 0, stream, F[2], nl, R, lam, c.ctrl, info);
  GLINT_LAUNCHED("k_absorb");
  return GLINT_OK;
}

template <int R>
glint_status texel_mttkrp(const glint_ndf_desc* d, const float* nxy, int mode, const double* const F[5], double* M,
                          unsigned char* ws, const TexelLayout& Lo, hipStream_t stream) {
  TexelCtx c;
  texel_ctx(d, nxy, Lo, ws, M, stream, &c);
  glint_status st = glint_texel_bins(d, nxy, c.bins, c.mass, stream);
  if (st != GLINT_OK) return st;
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, stream, c.ctrl);
  c.R = R;
  texel_zero_padding(c);
  texel_window<R>(c, F[0], d->nu, c.ub);
  texel_window<R>(c, F[1], d->nv, c.vb);
  if (mode <= 2) texel_p<R>(c, F[3], F[4]);
  else texel_w<R>(c, F[2]);
  GLINT_LAUNCHED("texel MTTKRP set-up");
  return texel_mode<R>(c, mode, F[2], F[3], F[4]);
}

glint_status check_texel_args(const glint_ndf_desc* d, const float* nxy, int R, void* ws, size_t ws_bytes,
                              TexelLayout* Lo) {
  glint_status st = glint_check_desc(d);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(nxy && ws, "null pointer argument");
  GLINT_SUPPORT(R == 16 || R == 32 || R == 64 || R == 128 || R == 256, "rank %d not in {16,32,64,128,256}", R);
  GLINT_REQUIRE(glint_aligned(ws, 256), "workspace must be 256-byte aligned");
  GLINT_REQUIRE(glint_aligned(nxy, 8), "nxy must be 8-byte aligned");
  texel_layout(d, R, Lo);
  if (ws_bytes < Lo->total)
    return glint_fail(GLINT_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, Lo->total);
  int dev = 0, max_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return glint_fail(GLINT_E_HIP, "hipDeviceGetAttribute failed");
  const int RT = R < 64 ? R : 64;
  if (static_cast<size_t>(max_lds) < sizeof(double) * 2 * d->nbins * RT)
    return glint_fail(GLINT_E_UNSUPPORTED, "texel tiles of %d bins do not fit in LDS (%d bytes)", d->nbins, max_lds);
  return GLINT_OK;
}

}  // namespace

extern "C" {

glint_status glint_mttkrp(const glint_ndf_desc* desc, const void* T, glint_dtype T_dtype, int32_t R,
                          int32_t mode, const double* U, const double* V, const double* L,
                          const double* S, const double* Tf, double* M, void* workspace,
                          size_t workspace_bytes, hipStream_t stream) {
  AlsLayout Lo;
  glint_status st = check_als_args(desc, T, T_dtype, R, workspace, workspace_bytes, &Lo);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(mode >= 0 && mode <= 4, "mode %d outside 0..4", mode);
  GLINT_REQUIRE(U && V && L && S && Tf && M, "null pointer argument");
  const double* F[5] = {U, V, L, S, Tf};
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  auto go = [&](auto ttag) -> glint_status {
    using TT = decltype(ttag);
    const TT* Tp = static_cast<const TT*>(T);
    switch (R) {
      case 16: return run_mttkrp<TT, 16>(desc, Tp, mode, F, M, ws, Lo, stream);
      case 32: return run_mttkrp<TT, 32>(desc, Tp, mode, F, M, ws, Lo, stream);
      case 64: return run_mttkrp<TT, 64>(desc, Tp, mode, F, M, ws, Lo, stream);
      default: return run_mttkrp<TT, 128>(desc, Tp, mode, F, M, ws, Lo, stream);
    }
  };
  if (T_dtype == GLINT_F64) return go(double{});
  return go(float{});
}

size_t glint_cp_als_workspace(const glint_ndf_desc* desc, int32_t R, glint_dtype T_dtype) {
  if (glint_check_desc(desc) != GLINT_OK) return 0;
  if (R < 16 || R > 128 || !glint_pow2(R)) return 0;
  if (T_dtype != GLINT_F64 && T_dtype != GLINT_F32) return 0;
  AlsLayout L;
  als_layout(desc, R, glint_dtype_size(T_dtype), &L);
  return L.total;
}

glint_status glint_cp_als(const glint_ndf_desc* desc, const void* T, glint_dtype T_dtype, int32_t R,
                          int32_t iters, double tol, double* U, double* V, double* L, double* S,
                          double* Tf, double* fit_hist, int32_t* info, void* workspace,
                          size_t workspace_bytes, hipStream_t stream) {
  AlsLayout Lo;
  glint_status st = check_als_args(desc, T, T_dtype, R, workspace, workspace_bytes, &Lo);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(U && V && L && S && Tf && fit_hist, "null pointer argument");
  GLINT_REQUIRE(iters >= 1, "iters must be >= 1");
  GLINT_REQUIRE(tol >= 0.0, "tol must be >= 0");
  double* F[5] = {U, V, L, S, Tf};
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  auto go = [&](auto ttag) -> glint_status {
    using TT = decltype(ttag);
    const TT* Tp = static_cast<const TT*>(T);
    switch (R) {
      case 16: return run_als<TT, 16>(desc, Tp, iters, tol, F, fit_hist, info, ws, Lo, stream);
      case 32: return run_als<TT, 32>(desc, Tp, iters, tol, F, fit_hist, info, ws, Lo, stream);
      case 64: return run_als<TT, 64>(desc, Tp, iters, tol, F, fit_hist, info, ws, Lo, stream);
      default: return run_als<TT, 128>(desc, Tp, iters, tol, F, fit_hist, info, ws, Lo, stream);
    }
  };
  if (T_dtype == GLINT_F64) return go(double{});
  return go(float{});
}

size_t glint_cp_als_texel_workspace(const glint_ndf_desc* desc, int32_t R) {
  if (glint_check_desc(desc) != GLINT_OK) return 0;
  if (!(R == 16 || R == 32 || R == 64 || R == 128 || R == 256)) return 0;
  TexelLayout L;
  texel_layout(desc, R, &L);
  return L.total;
}

glint_status glint_mttkrp_texel(const glint_ndf_desc* desc, const float* nxy, int32_t R, int32_t mode,
                                const double* U, const double* V, const double* L, const double* S,
                                const double* Tf, double* M, void* workspace, size_t workspace_bytes,
                                hipStream_t stream) {
  TexelLayout Lo;
  glint_status st = check_texel_args(desc, nxy, R, workspace, workspace_bytes, &Lo);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(mode >= 0 && mode <= 4, "mode %d outside 0..4", mode);
  GLINT_REQUIRE(U && V && L && S && Tf && M, "null pointer argument");
  const double* F[5] = {U, V, L, S, Tf};
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  switch (R) {
    case 16: return texel_mttkrp<16>(desc, nxy, mode, F, M, ws, Lo, stream);
    case 32: return texel_mttkrp<32>(desc, nxy, mode, F, M, ws, Lo, stream);
    case 64: return texel_mttkrp<64>(desc, nxy, mode, F, M, ws, Lo, stream);
    case 128: return texel_mttkrp<128>(desc, nxy, mode, F, M, ws, Lo, stream);
    default: return texel_mttkrp<256>(desc, nxy, mode, F, M, ws, Lo, stream);
  }
}

glint_status glint_cp_als_texel(const glint_ndf_desc* desc, const float* nxy, int32_t R, int32_t iters,
                                double tol, double normT2, double* U, double* V, double* L, double* S,
                                double* Tf, double* fit_hist, int32_t* info, void* workspace,
                                size_t workspace_bytes, hipStream_t stream) {
  TexelLayout Lo;
  glint_status st = check_texel_args(desc, nxy, R, workspace, workspace_bytes, &Lo);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(U && V && L && S && Tf && fit_hist, "null pointer argument");
  GLINT_REQUIRE(iters >= 1, "iters must be >= 1");
  GLINT_REQUIRE(tol >= 0.0, "tol must be >= 0");
  GLINT_REQUIRE(tol == 0.0 || normT2 > 0.0, "tol > 0 needs normT2 > 0");
  double* F[5] = {U, V, L, S, Tf};
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  switch (R) {
    case 16: return run_texel_als<16>(desc, nxy, iters, tol, normT2, F, fit_hist, info, ws, Lo, stream);
    case 32: return run_texel_als<32>(desc, nxy, iters, tol, normT2, F, fit_hist, info, ws, Lo, stream);
    case 64: return run_texel_als<64>(desc, nxy, iters, tol, normT2, F, fit_hist, info, ws, Lo, stream);
    case 128: return run_texel_als<128>(desc, nxy, iters, tol, normT2, F, fit_hist, info, ws, Lo, stream);
    default: return run_texel_als<256>(desc, nxy, iters, tol, normT2, F, fit_hist, info, ws, Lo, stream);
  }
}

}  // extern "C"
