/*
 * glint.h -- C ABI of libglint: constant-cost spatio-angular range queries of
 * a glint P-NDF compressed by CP (tensor-rank) decomposition, on AMD gfx950.
 *
 * Method: Deng et al., "Constant-Cost Spatio-Angular Prefiltering of Glinty
 * Appearance Using Tensor Decomposition".  Sec. 3.1 (Eq. geom) defines the
 * P-NDF, Sec. 4.1 the footprint pyramid over every texel and level, Sec. 4.2
 * (Eq. compress) the CP fit by alternating least squares, Sec. 4.3
 * (Eq. decompress) the point query and Sec. 4.4 (Eq. rangeDecom, summed-area
 * tables, and the Appendix proposition) the constant-cost range query.
 *
 * Conventions for every call:
 *   - Pointers are DEVICE pointers unless a parameter says "host".  The caller
 *     owns every buffer (inputs, outputs, workspace); the library allocates
 *     nothing and keeps no state between calls.
 *   - Each call validates its arguments on the host and returns a status
 *     synchronously; on success the work is enqueued on `stream` and the call
 *     returns without waiting.  A failed kernel launch returns GLINT_E_HIP.
 *     Faults inside kernels surface at the caller's next synchronisation.
 *   - glint_last_error() gives a human-readable detail of the last non-OK
 *     status returned on the calling thread.
 *   - Tensors are row-major; "[a][b]" means b is the fastest index.
 *   - No call throws across the ABI.
 *
 * Query records are int32 [7] = (u, v, l, s_lo, s_hi, t_lo, t_hi): footprint
 * centre (u, v), level l (a 2^l x 2^l texel box), and half-open bin ranges
 * [s_lo, s_hi) x [t_lo, t_hi).  Index rules (kernels never fault on them):
 * u, v wrap modulo the map size (maps are tileable); l clamps to
 * [0, nlevels-1] (footprints beyond the pyramid clamp to its coarsest level,
 * Sec. 5.1); bin bounds clamp to [0, nbins]; a box with lo >= hi on either
 * axis gives exactly 0.  The value returned is the box SUM of bin masses;
 * the paper's box average is sum / ((s_hi - s_lo) * (t_hi - t_lo)).
 */
#ifndef GLINT_H
#define GLINT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t glint_status;
#define GLINT_OK             0
#define GLINT_E_INVALID     (-1)   /* bad argument: null pointer, size, alignment */
#define GLINT_E_UNSUPPORTED (-2)   /* valid but not implemented (dtype, rank, size) */
#define GLINT_E_HIP         (-3)   /* a HIP runtime call or kernel launch failed */
#define GLINT_E_WORKSPACE   (-4)   /* workspace smaller than the *_workspace size */

typedef enum glint_dtype {
  GLINT_F64 = 0,
  GLINT_F32 = 1,
  GLINT_BF16 = 2,       /* bfloat16, stored as uint16 bit patterns */
  GLINT_FP8E4M3 = 3     /* OCP E4M3FN, stored as uint8, with per-column FP32 scales */
} glint_dtype;

/* The NDF tensor T[u][v][l][s][t] of a normal map (Sec. 3.1, Sec. 4.1).
 * A texel with projected normal (n_x, n_y) contributes m_x[s] * m_y[t] to bin
 * (s, t), where m_x[i] is the mass of a Gaussian of standard deviation sigma
 * centred on n_x inside bin i, edges e_i = -1 + 2i/N, renormalised to the mass
 * inside [-1, 1].  Level l averages the texels of the box of side k = 2^l
 * anchored at (u - k/2, v - k/2) (integer division), wrapping. */
typedef struct glint_ndf_desc {
  int32_t nu, nv;       /* normal-map size in texels (u slow, v fast), >= 1 */
  int32_t nlevels;      /* footprint levels, 1..16; 2^(nlevels-1) <= min(nu, nv) */
  int32_t nbins;        /* N: bins per axis over [-1, 1]; power of two, 4..256 */
  double sigma;         /* intrinsic roughness, > 0 */
} glint_ndf_desc;

/* Compressed factors for the range query (Sec. 4.4, Eq. rangeDecom):
 *   q = sum_r c[r] * U[u][r] V[v][r] L[l][r] (CS[s_hi][r] - CS[s_lo][r])
 *                                         (CT[t_hi][r] - CT[t_lo][r]),
 * values decoded exactly from their storage type, and c[r] the product (FP32,
 * in the order U, V, L, CS, CT) of the per-column scales given (a NULL scale
 * is 1).  CS, CT are the 1D summed-area tables of the S and T factors:
 * CS[j][r] = sum_{s<j} S[s][r], j = 0..nbins. */
typedef struct glint_factors {
  int32_t R;            /* rank: 16, 32, 64, 128 or 256 */
  int32_t nu, nv, nl;   /* rows of U, V, L */
  int32_t nbins;        /* N; CS and CT have N+1 rows */
  glint_dtype dtype;    /* storage of U, V, L: F32, BF16 or FP8E4M3 */
  glint_dtype cum_dtype;/* storage of CS, CT: F32, BF16 or FP8E4M3 */
  const void* U;        /* [nu][R], 16-byte aligned */
  const void* V;        /* [nv][R] */
  const void* L;        /* [nl][R] */
  const void* CS;       /* [N+1][R] */
  const void* CT;       /* [N+1][R] */
  const float* scale_U; /* [R] per-column scale of U (FP8 storage), or NULL */
  const float* scale_V;
  const float* scale_L;
  const float* scale_CS;
  const float* scale_CT;
} glint_factors;

/* ---- identification ------------------------------------------------------ */
const char* glint_status_string(glint_status s);
const char* glint_last_error(void);
int32_t glint_version(void);

/* ---- step 1: per-texel angular binning (Sec. 3.1, Eq. geom) --------------- */

/* Half-width K of the per-texel bin window: K = ceil(8 sigma / w) + 1 with
 * w = 2/N.  Bins further than K from a texel's centre bin hold less than
 * Phi(-8) of its mass and are treated as 0.  Returns -1 for an invalid desc. */
int32_t glint_window_radius(const glint_ndf_desc* desc);

/* For every texel (u, v) and axis a (0: s from n_x, 1: t from n_y):
 *   bins[(u*nv + v)*2 + a] = i0 = clamp(floor((n + 1) * N/2), 0, N-1), in FP64;
 *   mass[((u*nv + v)*2 + a)*(2K+1) + j] = normalised mass of bin i0 - K + j
 *     (0 where that bin is outside [0, N)).
 * nxy: [nu][nv][2] float32 projected normals.  bins: int32, mass: double.
 * A non-finite component marks the axis of an absent texel: bin 0 and all
 * masses 0, so the texel contributes nothing to the tensor, the range
 * integrals or the texel-space ALS (Wang tiles pad a tile with absent texels,
 * Sec. 5.5). */
glint_status glint_texel_bins(const glint_ndf_desc* desc, const float* nxy,
                              int32_t* bins, double* mass, hipStream_t stream);

/* ---- step 2: NDF tensor over every texel and level (Sec. 4.1) ------------ */

/* Workspace bytes for glint_build_tensor (the bin windows). */
size_t glint_build_tensor_workspace(const glint_ndf_desc* desc);

/* T[u][v][l][s][t] (dtype F64 or F32), every entry written.  Levels
 * l < direct_levels are built directly from their footprint texels (the
 * texels' bin windows staged in LDS); each higher level is the exact mean of
 * four shifted blocks of the level below (a 2k box is two k boxes per axis).
 * direct_levels <= 0 selects the default (3: above it the direct build's
 * LDS accumulation of k^2 overlapping texel windows costs more than a
 * doubling pass, measured on the 512^2 map); values above nlevels mean
 * "every level directly".  T must be 16-byte aligned. */
glint_status glint_build_tensor(const glint_ndf_desc* desc, const float* nxy,
                                void* T, glint_dtype T_dtype, int32_t direct_levels,
                                void* workspace, size_t workspace_bytes,
                                hipStream_t stream);

/* glint_build_tensor for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same kernels (the result equals glint_build_tensor's up to the order of
 * the direct build's LDS-atomic sums), with the bin windows kept in a scratch array
 * the library holds on each device it runs on (GLINT_NOALLOC_SCRATCH_BYTES,
 * held until the process ends) instead of a caller workspace.  Maps whose
 * glint_build_tensor_workspace exceeds that size return GLINT_E_UNSUPPORTED
 * before any work is enqueued (512 x 512 at K = 3 needs 31.5 MiB).  Calls no
 * allocating routine.  Every call on a device shares that device's scratch:
 * calls that overlap on one device (two streams, two threads) race; calls
 * in stream order are safe (every call overwrites what it reads). */
#define GLINT_NOALLOC_SCRATCH_BYTES (48u << 20)
glint_status glint_build_tensor_noalloc(const glint_ndf_desc* desc, const float* nxy,
                                        void* T, glint_dtype T_dtype, int32_t direct_levels,
                                        hipStream_t stream);

/* Brute-force range integral for the refinement targets and the error
 * against the exact NDF: out[i] = (1/k^2) sum over footprint texels of
 * (mass of the texel's s-window inside [s_lo, s_hi)) * (same for t), FP64.
 * bins, mass: output of glint_texel_bins for the same desc.  q: [nq][7]. */
glint_status glint_range_bruteforce(const glint_ndf_desc* desc, const int32_t* bins,
                                    const double* mass, int64_t nq, const int32_t* q,
                                    double* out, hipStream_t stream);

/* ---- step 3: CP decomposition by ALS (Sec. 4.2, Eq. compress) ------------ */

/* Workspace bytes for glint_cp_als on a materialised T of this desc. */
size_t glint_cp_als_workspace(const glint_ndf_desc* desc, int32_t R, glint_dtype T_dtype);

/* Rank-R CP-ALS of T (dtype F64: FP64 matrix-core MTTKRP; F32: FP32
 * matrix-core MTTKRP).  Factors are FP64 [rows][R] in/out: on entry the
 * initial factors, on exit the fit with unit-norm columns in U, V, S, Tf and
 * the column weights lambda absorbed into L.  Each sweep updates the modes in
 * the order u, v, l, s, t; a mode update is A_n = M_n G^-1 with the Gram
 * Hadamard product G factored by FP64 Cholesky.  fit_hist[iters] receives
 * 1 - ||T - T^|| / ||T|| after each sweep (sweeps skipped after convergence
 * repeat the last value).  If tol > 0 the sweeps stop once the fit changes by
 * less than tol.  info (int32[4], may be NULL): sweeps run, mode updates whose
 * Cholesky broke down (a pivot not above 1e-13 times its diagonal entry of
 * G), and two reserved zeros.  Such an update takes A_n = M_n G+ instead,
 * G+ the eigen pseudo-inverse of G with the eigenvalues not above 1e-12
 * times the largest dropped (cyclic Jacobi on one workgroup, using the
 * workspace's Cholesky buffers).  R in {16, 32, 64, 128}; nbins >= 16. */
glint_status glint_cp_als(const glint_ndf_desc* desc, const void* T, glint_dtype T_dtype,
                          int32_t R, int32_t iters, double tol,
                          double* U, double* V, double* L, double* S, double* Tf,
                          double* fit_hist, int32_t* info,
                          void* workspace, size_t workspace_bytes, hipStream_t stream);

/* The MTTKRP of one mode, the contraction a mode update of glint_cp_als
 * starts from: M[i][r] = sum over the other four indices of T times the
 * product of the other four factors' entries in column r.  mode: 0 u, 1 v,
 * 2 l, 3 s, 4 t.  Uses the same matrix-core passes as glint_cp_als (the
 * (s,t) contraction pass for modes u, v, l; the cell contraction pass for
 * modes s, t).  Factors FP64 [rows][R], M FP64 [rows of the mode][R];
 * workspace of glint_cp_als_workspace bytes; same limits as glint_cp_als. */
glint_status glint_mttkrp(const glint_ndf_desc* desc, const void* T, glint_dtype T_dtype,
                          int32_t R, int32_t mode, const double* U, const double* V,
                          const double* L, const double* S, const double* Tf, double* M,
                          void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Texel-space forms of the two calls above, for maps whose tensor T does not
 * fit in memory.  T (Sec. 3.1, Eq. geom, over the footprint pyramid of
 * Sec. 4.1 with the square footprints of glint_ndf_desc) is the footprint
 * average of per-texel outer products of the s-
 * and t-bin masses, so each MTTKRP is evaluated from the per-texel bin
 * windows of glint_texel_bins and window sums of U and V over the footprint
 * pyramid; T is never formed.  The results equal those of glint_mttkrp /
 * glint_cp_als on the materialised FP64 T up to FP64 rounding order.
 * nxy: float [nu][nv][2] normal map (as for glint_build_tensor), 8-byte
 * aligned.  All arithmetic FP64.  R in {16, 32, 64, 128, 256}; nbins <= 128
 * when R >= 64 (two [nbins][64] FP64 tiles must fit in one block's LDS),
 * else any valid desc.
 * Workspace: glint_cp_als_texel_workspace bytes, 256-byte aligned; it holds
 * three FP64 [nu*nv][R] texel arrays, so it grows with the map, not with
 * the tensor. */
size_t glint_cp_als_texel_workspace(const glint_ndf_desc* desc, int32_t R);

/* Texel-space MTTKRP of one mode (0 u, 1 v, 2 l, 3 s, 4 t); M FP64
 * [rows of the mode][R]; factors FP64 [rows][R]. */
glint_status glint_mttkrp_texel(const glint_ndf_desc* desc, const float* nxy, int32_t R,
                                int32_t mode, const double* U, const double* V,
                                const double* L, const double* S, const double* Tf,
                                double* M, void* workspace, size_t workspace_bytes,
                                hipStream_t stream);

/* Texel-space CP-ALS: same sweep order, update rule, breakdown rule, factor
 * normalisation and outputs as glint_cp_als.  ||T||^2 is not computable
 * without T, so the caller supplies normT2 (host double); if normT2 <= 0 the
 * fit history is NaN and tol must be 0. */
glint_status glint_cp_als_texel(const glint_ndf_desc* desc, const float* nxy, int32_t R,
                                int32_t iters, double tol, double normT2,
                                double* U, double* V, double* L, double* S, double* Tf,
                                double* fit_hist, int32_t* info,
                                void* workspace, size_t workspace_bytes, hipStream_t stream);

/* ---- clustered layout (Sec. 4.2, Eq. compress and its practical choices) --
 * Each NDF image is cut into t x t angular blocks and footprints are grouped
 * by the cs x cs texel region of their centre; the blocks of one region and
 * one angular position form a 3-way tensor D[a][b][f] (a, b the bins inside
 * the block, f = (du * cs + dv) * nlevels + l for the centre
 * (cu * cs + du, cv * cs + dv)), fitted by its own rank-R CP.
 * Tensor index = ((cu * ncv + cv) * nb + zs) * nb + zt with ncv = nv / cs,
 * nb = nbins / t. */
typedef struct {
  int32_t t;    /* angular block side in bins (min(t, nbins) is used; must divide nbins; <= 16) */
  int32_t cs;   /* region side in texels (divides nu and nv) */
  int32_t R;    /* rank per region-and-block tensor: 4, 8, 16 or 32 */
} glint_cluster_desc;

/* CP-ALS of every region-and-block tensor of T (F64 or F32, the layout of
 * glint_build_tensor), one workgroup per tensor, FP64 arithmetic.  Blank
 * image blocks are thrown away first (Sec. 4.2): the block of footprint f
 * is blank when the sum of its |values| is <= 1e-12, and only the L'
 * non-blank blocks are stacked (in footprint order) and fitted; a blank
 * footprint's Z row is zero.  A tensor with L' = 0 is blank: zero factors,
 * blank[tensor] = 1, counted in info[1].  Modes X (a), Y (b), Z (f) in that
 * order, `iters` sweeps; normal equations with a ridge: A = M (G + mu I)^-1,
 * mu = 1e-10 trace(G) / R, by Cholesky; a pivot <= 1e-13 times its diagonal
 * entry keeps that mode's factor for the sweep (counted in info[0]).
 * Columns unit after each update; their weights end in Z.  Initial factors
 * U[0,1) from SplitMix64 used as a counter-based generator: value =
 * (mix(seed + (c + 1) * 0x9E3779B97F4A7C15) >> 11) 2^-53,
 * c = ((tensor * 3 + mode) * max(t, L) + row) * R + r, where the row of a Z
 * entry is its footprint f.  Outputs FP32: X, Y [ntensor][t][R],
 * Z [ntensor][L][R] with L = cs * cs * nlevels; blank uint8 [ntensor];
 * info int32 [4]: failures, blank tensors, the call's work counter, and the
 * total L' over all tensors (the stacked blocks, for the compression
 * ratio).  The tensor's factors, Grams and partial products live in LDS for
 * all sweeps: configurations that do not fit return GLINT_E_UNSUPPORTED
 * (rank 16 fits with t = 16, cs = 8 and up to 8 levels from an F32 tensor). */
glint_status glint_cp_als_clustered(const glint_ndf_desc* desc, const glint_cluster_desc* cd,
                                    const void* T, glint_dtype T_dtype, int32_t iters,
                                    uint64_t seed, float* X, float* Y, float* Z,
                                    uint8_t* blank, int32_t* info, hipStream_t stream);

/* The clustered layout of a normal map whose tensor T is not stored (Sec. 4.2
 * practical choices at the paper's scale: t = 16, 8 x 8 texel regions, rank
 * 16 or 32, every level).  The angular blocks are taken one at a time: the
 * tensor of one block, T restricted to bins [zs t, zs t + t) x [zt t, zt t +
 * t) for every texel and level, is built in the workspace from the texel bin
 * windows (as glint_build_tensor builds T: level 0 directly, each higher
 * level the exact mean of four shifted blocks of the level below), in
 * T_dtype (F32 or F64), and its region tensors are fitted there.  Factors,
 * blank rule, ALS, initial factors and outputs X, Y, blank, info are those
 * of glint_cp_als_clustered for the same tensor; Z is stored compactly:
 * only the non-blank footprints' rows, at the rows zidx names.  Where the Z
 * factors of a tensor do not fit the LDS (rank 32 with 320 or more
 * footprints) they live in the workspace (one slot per running workgroup).
 * Two calls in stream order:
 *  - glint_cluster_map_index fills zidx int32 [ntensor][L] (the footprint's
 *    row of Z or -1 for a blank image block; rows numbered tensor by tensor,
 *    footprints in order) and zbase int64 [ntensor + 1] (the first row of
 *    each tensor; zbase[ntensor] = the number of rows, which the caller
 *    reads to size Z); info as for glint_cp_als_clustered (info[1] blank
 *    tensors, info[3] rows).
 *  - glint_cp_als_clustered_map fits every tensor and writes X, Y
 *    [ntensor][t][R], Z [rows][R] (weights absorbed), blank [ntensor], info.
 * Rows must stay below 2^31.  The workspace (glint_cluster_map_workspace
 * bytes, 256-byte aligned; the block tensor takes nu nv nlevels t^2
 * elements of T_dtype) is the same for both calls; the workspace size
 * depends on the device's CU count. */
size_t glint_cluster_map_workspace(const glint_ndf_desc* desc, const glint_cluster_desc* cd, glint_dtype T_dtype);
glint_status glint_cluster_map_index(const glint_ndf_desc* desc, const glint_cluster_desc* cd, const float* nxy,
                                     glint_dtype T_dtype, int32_t* zidx, int64_t* zbase, int32_t* info,
                                     void* workspace, size_t workspace_bytes, hipStream_t stream);
glint_status glint_cp_als_clustered_map(const glint_ndf_desc* desc, const glint_cluster_desc* cd, const float* nxy,
                                        glint_dtype T_dtype, int32_t iters, uint64_t seed, const int32_t* zidx,
                                        float* X, float* Y, float* Z, uint8_t* blank, int32_t* info,
                                        void* workspace, size_t workspace_bytes, hipStream_t stream);

/* C[b][j][r] = sum_{s<j} S[b][s][r] (FP64 accumulation, FP32 out) for
 * nbatch stacked [n][R] tables; C is [nbatch][n+1][R]. */
glint_status glint_make_cumulative_batched(int64_t nbatch, int32_t n, int32_t R, const float* S,
                                           float* C, hipStream_t stream);

/* Clustered query tables: summed-area tables of X and Y per tensor,
 * CX, CY [ntensor][t+1][R], and Z: dense [ntensor][L][R] (zidx NULL) or,
 * in the compact layout, [rows][R] with zidx [ntensor][L] giving each
 * footprint's row of Z, -1 for a blank image block (no terms); 16-byte
 * aligned.  dtype is the element type of CX, CY and Z: GLINT_F32, or
 * GLINT_BF16 (Sec. 4.4 storage: each FP32 table value rounded to nearest
 * even, as glint_convert does; half the gathered bytes), read by
 * glint_query_clustered only; any other value is GLINT_E_INVALID. */
typedef struct {
  int32_t t, cs, R;
  int32_t nu, nv, nl, nbins;
  const void* CX;
  const void* CY;
  const void* Z;
  const int32_t* zidx;
  int32_t dtype;
} glint_clustered;

/* Range query on the clustered tables: records as for glint_query (same
 * wrap/clamp/empty rules); the box is split at block edges and the
 * block-local queries sum_r Z[f][r] (CX[a1][r] - CX[a0][r]) (CY[b1][r] -
 * CY[b0][r]) are added (a blank image block of the compact layout adds
 * nothing).  FP32 arithmetic on the stored values (BF16 tables decoded
 * exactly to FP32). */
glint_status glint_query_clustered(const glint_clustered* f, int64_t nq, const int32_t* q,
                                   float* out, hipStream_t stream);

/* Hierarchical importance sampling on the clustered tables (Sec. 5.2: start
 * from an image block chosen by the blocks' masses, then descend by quads):
 * for lookup i (uvl [n][3], wrapped/clamped as for queries) with draws
 * rnd [n][log2(t) + 3] in [0, 1): the block by rnd[0] among the nb x nb
 * blocks in zs-major order with probability proportional to its mass (the
 * block-local query over the whole block, negative masses as zero; the
 * draw picks the first block whose running mass exceeds rnd[0] times the
 * total, never an empty one), then log2(t) levels of four quads, (s lo,
 * t lo), (s lo, t hi), (s hi, t lo), (s hi, t hi), by rnd[1..log2 t] with
 * the same rule, then h = (-1 + (s + rnd[log2 t + 1]) 2/N, -1 + (t +
 * rnd[log2 t + 2]) 2/N) with (s, t) the global bin; pdf = the product of
 * the choice probabilities / (2/N)^2.  No positive mass: bins (-1, -1),
 * pdf 0, h 0.  t must be a power of two.  Outputs h float [n][2], pdf float
 * [n], bins int32 [n][2].  One thread per lookup, FP32; FP32 tables only
 * (dtype GLINT_F32, else GLINT_E_UNSUPPORTED). */
glint_status glint_sample_clustered(const glint_clustered* f, int64_t n, const int32_t* uvl, const float* rnd,
                                    float* h, float* pdf, int32_t* bins, hipStream_t stream);

/* ---- step 4: summed-area tables and storage types (Sec. 4.4) ------------ */

/* C[j][r] = sum_{s<j} S[s][r] for j = 0..n, accumulated in FP64 and then
 * stored as out_dtype: F64, F32 (round to nearest even from FP64), BF16
 * (FP64 -> FP32 -> BF16, each round to nearest even) or FP8E4M3 (per-column
 * scale = amax/448 of the FP32 values, code = RNE(x/scale), saturating; the
 * scales go to col_scale[R], which must then be non-NULL).
 * S: [n][R] of dtype in_dtype (F64 or F32).  C: [n+1][R]. */
glint_status glint_make_cumulative(int32_t n, int32_t R, const void* S, glint_dtype in_dtype,
                                   void* C, glint_dtype out_dtype, float* col_scale,
                                   hipStream_t stream);

/* Storage conversion of a factor table [rows][R]: in F64 or F32; out F32,
 * BF16 or FP8E4M3 (per-column scales as in glint_make_cumulative, written to
 * col_scale). */
glint_status glint_convert(int64_t rows, int32_t R, const void* in, glint_dtype in_dtype,
                           void* out, glint_dtype out_dtype, float* col_scale,
                           hipStream_t stream);

/* ---- step 5: the range query (Sec. 4.4, Eq. rangeDecom; Appendix) ------- */

/* out[i] for each record q[i] (int32 [nq][7], see the header comment), FP32
 * arithmetic on values decoded exactly from their storage types.
 * nq = 0 is a no-op.  Requires f->nbins in 4..256, f->nu <= 2^26 and
 * f->nl <= 64 (records are resolved into 16-byte packed rows; larger maps
 * or level counts return GLINT_E_UNSUPPORTED before any launch).  L is
 * staged in LDS as FP32 (nl * R * 4 bytes); CS and CT are staged there too
 * (as FP32, or as BF16 when so stored beyond rank 64) when they fit, and
 * otherwise read from global memory. */
glint_status glint_query(const glint_factors* f, int64_t nq, const int32_t* q,
                         float* out, hipStream_t stream);

/* Grouped form for shading points that share a footprint: uvl int32
 * [npts][3] = (u, v, l), boxes int32 [npts][K][4] = (s_lo, s_hi, t_lo, t_hi),
 * out float [npts][K].  Same value as glint_query on the expanded records. */
glint_status glint_query_grouped(const glint_factors* f, int64_t npts, int32_t K,
                                 const int32_t* uvl, const int32_t* boxes,
                                 float* out, hipStream_t stream);

/* Off-grid footprints (Sec. 4.1 and Sec. 4.3): the trilinear blend of the
 * range queries of the eight precomputed footprints around a continuous
 * centre and level.  xyl: float [nq][3] = (x, y, lam) in index units (the
 * corners are floor(x) and floor(x)+1, wrapping; likewise y; floor(lam) and
 * floor(lam)+1 with lam clamped to [0, nl-1]); a non-finite coordinate
 * counts as 0 and |x|, |y| are clamped to 2^24.  boxes: int32 [nq][4] =
 * (s_lo, s_hi, t_lo, t_hi) with the clamping and empty-box rules of
 * glint_query.  Evaluated as one query with linearly interpolated U, V and
 * L rows (the reconstruction is multilinear, so this equals the blend),
 * FP32 arithmetic; same table limits as glint_query. */
glint_status glint_query_trilinear(const glint_factors* f, int64_t nq, const float* xyl,
                                   const int32_t* boxes, float* out, hipStream_t stream);

/* Hierarchical importance sampling of a footprint's NDF image by range
 * queries (Sec. 5.2).  For each record uvl[i] = (u, v, l) (wrapped/clamped
 * as in glint_query): the N x N image is split into four quads, ordered
 * (s low, t low), (s low, t high), (s high, t low), (s high, t high); quad
 * masses are range queries, negative ones count as zero; the draw
 * rnd[i][k] in [0, 1) picks the first quad whose running mass sum exceeds
 * rnd * total; this repeats for log2(N) levels, then
 * h[i] = (-1 + (s + rnd[i][L]) * 2/N, -1 + (t + rnd[i][L+1]) * 2/N) with
 * L = log2(N) and (s, t) = bins[i] the final bin; pdf[i] = P(bin) / (2/N)^2,
 * P(bin) the product of the chosen quads' probabilities (the normalised
 * NDF mass of the bin when no mass is negative).  A record whose quads hold
 * no positive mass at some level gets bins (-1, -1), pdf 0, h (0, 0).
 * rnd: float [n][L + 2] (the caller's uniform draws); h: float [n][2];
 * pdf: float [n]; bins: int32 [n][2].  FP32 arithmetic; same table limits
 * as glint_query. */
glint_status glint_sample(const glint_factors* f, int64_t n, const int32_t* uvl, const float* rnd,
                          float* h, float* pdf, int32_t* bins, hipStream_t stream);

/* Counts the records the query's rules would change (for callers that want
 * errors instead of wrapping and clamping): u or v outside the map, l
 * outside [0, nl), a bin bound outside [0, N], or a reversed box (lo > hi;
 * lo == hi is a valid empty box).  nbad: one device int64, overwritten
 * (cleared by a small kernel, so the call can be captured in a graph).
 * Only the table sizes of f are used. */
glint_status glint_validate_queries(const glint_factors* f, int64_t nq, const int32_t* q, int64_t* nbad,
                                    hipStream_t stream);

/* Environment-light prefiltering (Sec. 5.4, compact-eps support and the box
 * side Q): for lookup i with footprint uvl[i] = (u, v, l), projected half
 * vector h[i] = (h_s, h_t) in [-1, 1]^2 and the spherical-Gaussian light
 * lobe sg[i] = (lambda, A) chosen for it, theta = arccos(clamp((ln eps -
 * ln A) / lambda + 1, -1, 1)) (FP64) and the square of side
 * w = min(2 theta / pi, 2) (N theta / pi bins) centred on h gives the bins
 * lo = clamp(floor((h - w/2 + 1) N/2), 0, N-1),
 * hi = clamp(floor((h + w/2 + 1) N/2), 0, N-1) + 1 per axis (at least one
 * bin: a zero-width box is the point lookup of the bin holding h).  The
 * records are written to q [n][7] (the glint_query layout, for reuse, e.g.
 * by the backward), and out[i] = the box sum / its number of bins, the
 * average bin mass.  A non-finite h component counts as 0; a lobe whose
 * argument is not finite (lambda = 0, A <= 0) gives the point lookup.  eps
 * (0.3 in the paper) must be finite and positive.  Other rules as
 * glint_query. */
glint_status glint_query_sg(const glint_factors* f, int64_t n, const int32_t* uvl, const float* h,
                            const float* sg, float eps, int32_t* q, float* out, hipStream_t stream);

/* Wang tiles (Sec. 5.5): constant-storage synthesis of an unbounded normal
 * map.  The plane is a grid of S x S cells; cell (i, j) holds the plane
 * texels x in [iS, (i+1)S), y in [jS, (j+1)S).  Vertex (i, j) colours the
 * edge to its right (e = 0) and the edge below it (e = 1) with
 * colour = [SplitMix64 U[0,1) >= 1/2] at counter
 * ((((i mod 2^32) << 32) | (j mod 2^32)) << 1) | e (the generator of
 * glint_cp_als_clustered, seeded with `seed`); cell (i, j)'s tile is
 * edge_to_tile[8 top + 4 right + 2 bottom + left] with top = (i, j, 0),
 * right = (i+1, j, 1), bottom = (i, j+1, 0), left = (i, j, 1).  Each tile's
 * tables are a CP of the tensor of the tile padded with m absent texels
 * (non-finite normals, see glint_texel_bins) on every side: P = S + 2m rows
 * of U and V, padded index = tile index + m.  FP32 tables, stacked by tile:
 * U, V [ntiles][P][R], L [ntiles][nl][R], CS, CT [ntiles][N+1][R]. */
typedef struct {
  int32_t ntiles, S, m, R, nl, nbins;
  uint64_t seed;
  uint8_t edge_to_tile[16];   /* host copy, values < ntiles */
  const float* U;
  const float* V;
  const float* L;
  const float* CS;
  const float* CT;
} glint_wang;

/* Range queries on the synthesized plane: q [nq][7] = (x, y, l, s_lo, s_hi,
 * t_lo, t_hi) with plane texel coordinates (any int32, no wrap); l and the
 * bins clamp as for glint_query; out[i] = the sum, over the cells the level-l
 * footprint centred on (x, y) overlaps, of that cell's tile query at centre
 * (x - iS + m, y - jS + m).  Requires 2m >= 2^(nl-1) so every overlapped
 * cell's centre lies in its tile's padded grid, 2^(nl-1) <= S (tiles at
 * least as wide as the largest footprint, so a footprint overlaps at most
 * 2 x 2 cells and a query's work is bounded), R a multiple of 4 and the
 * tables 16-byte aligned.  One thread per query, FP32. */
glint_status glint_query_wang(const glint_wang* w, int64_t nq, const int32_t* q, float* out,
                              hipStream_t stream);

/* ---- step 6: gradient of the query (not in the paper) -------------------- */

/* Gradients of sum_i gout[i] * q[i] with respect to the stored values of U,
 * V, L, CS and CT (FP32, overwritten: the call clears them first).  f->dtype
 * and f->cum_dtype must be F32 or BF16.  dU [nu][R], dV [nv][R], dL [nl][R],
 * dCS, dCT [N+1][R].  Accumulation uses atomics, so the summation order (and
 * the last bits) vary between runs.  L, CS and CT are staged in LDS as FP32:
 * for N <= 64 (and nl <= 16) the summed-area-table and level gradients
 * accumulate on the matrix cores, needing 4 (nl + 2 (N + 1)) R + 4 R bytes
 * plus 32 KiB of record slots; for larger N their accumulators are held in
 * LDS as well (8 (nl + 2 (N + 1)) R + 4 R bytes plus 16 KiB).  Tables beyond
 * that return GLINT_E_UNSUPPORTED. */
glint_status glint_query_backward(const glint_factors* f, int64_t nq, const int32_t* q,
                                  const float* gout, float* dU, float* dV, float* dL,
                                  float* dCS, float* dCT, hipStream_t stream);

/* Chain rule through the summed-area table: dS[s][r] = sum_{j>s} dC[j][r].
 * dC: [n+1][R], dS: [n][R], FP32. */
glint_status glint_cumulative_backward(int32_t n, int32_t R, const float* dC, float* dS,
                                       hipStream_t stream);

/* ---- step 7: refinement helpers (not in the paper) ----------------------- */

/* Mean squared error against FP64 targets: loss[0] = (1/nq) sum (q - t)^2
 * (FP64), gout[i] = 2 (q[i] - t[i]) / nq (FP32).  loss may be NULL. */
glint_status glint_mse_grad(int64_t nq, const float* q, const double* target,
                            float* gout, double* loss, hipStream_t stream);

/* One Adam step (Kingma and Ba) on n FP32 parameters, step >= 1:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps). */
glint_status glint_adam_step(int64_t n, float* p, const float* g, float* m, float* v,
                             float lr, float b1, float b2, float eps, int32_t step,
                             hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* GLINT_H */
