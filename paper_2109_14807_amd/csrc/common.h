// Internal helpers shared by the libglint HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/glint.h"

// ---------------------------------------------------------------------------
// host-side status reporting
// ---------------------------------------------------------------------------

// Records a printf-style detail for glint_last_error() and returns `code`.
glint_status glint_fail(glint_status code, const char* fmt, ...);

#define GLINT_REQUIRE(cond, ...)                                   \
  do {                                                             \
    if (!(cond)) return glint_fail(GLINT_E_INVALID, __VA_ARGS__);  \
  } while (0)

#define GLINT_SUPPORT(cond, ...)                                       \
  do {                                                                 \
    if (!(cond)) return glint_fail(GLINT_E_UNSUPPORTED, __VA_ARGS__);  \
  } while (0)

// Checks the launch just made.  The error slot is cleared before each launch
// (glint_clear_launch_error) so that only this launch is reported.
#define GLINT_LAUNCHED(what)                                                        \
  do {                                                                              \
    hipError_t e_ = hipGetLastError();                                              \
    if (e_ != hipSuccess)                                                           \
      return glint_fail(GLINT_E_HIP, "%s: %s", (what), hipGetErrorString(e_));      \
  } while (0)

static inline void glint_clear_launch_error() { (void)hipGetLastError(); }

static inline bool glint_aligned(const void* p, size_t a) {
  return (reinterpret_cast<uintptr_t>(p) % a) == 0;
}

static inline bool glint_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

static inline int glint_log2(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

__host__ __device__ static inline size_t glint_round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static inline size_t glint_dtype_size(glint_dtype t) {
  switch (t) {
    case GLINT_F64: return 8;
    case GLINT_F32: return 4;
    case GLINT_BF16: return 2;
    case GLINT_FP8E4M3: return 1;
  }
  return 0;
}

// Validation of an NDF descriptor shared by the build, bins and ALS calls.
glint_status glint_check_desc(const glint_ndf_desc* d);

// Half-width of the per-texel bin window (see glint_window_radius).
int32_t glint_window_k(const glint_ndf_desc* d);

// The NDF tensor restricted to one window of bins: T[u][v][l][a][b] =
// the full tensor's entry at bins (s_off + a, t_off + b), a, b < nout, built
// from the texel bin windows of glint_texel_bins by the same kernels as
// glint_build_tensor (direct levels, then exact level doubling).  Library
// internal (the clustered layout builds its angular blocks this way).
glint_status glint_build_window(const glint_ndf_desc* desc, const int32_t* bins, const double* mass, void* T,
                                glint_dtype T_dtype, int32_t direct_levels, int32_t s_off, int32_t t_off,
                                int32_t nout, hipStream_t stream);

// ---------------------------------------------------------------------------
// device-side value codecs (written from the storage formats' definitions)
// ---------------------------------------------------------------------------

__device__ __forceinline__ float glint_bf16_to_f32(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

// FP32 -> BF16, round to nearest, ties to even; NaN stays a quiet NaN.
__device__ __forceinline__ uint16_t glint_f32_to_bf16(float x) {
  uint32_t b = __float_as_uint(x);
  if ((b & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;
  b += 0x7fffu + ((b >> 16) & 1u);
  return static_cast<uint16_t>(b >> 16);
}

// OCP E4M3FN code -> FP32 (bias 7, 3 mantissa bits, exponent 0 subnormal).
__device__ __forceinline__ float glint_fp8_to_f32(uint32_t c) {
  const uint32_t e = (c >> 3) & 0xfu;
  const uint32_t m = c & 7u;
  float v = (e == 0u) ? static_cast<float>(m) * 0.001953125f           // m * 2^-9
                      : __uint_as_float(((c & 0x7fu) << 20) + 0x3c000000u);  // rebias 7 -> 127
  if (e == 15u && m == 7u) v = __uint_as_float(0x7fc00000u);
  return (c & 0x80u) ? -v : v;
}

// FP32 -> OCP E4M3FN, round to nearest, ties to even, saturating at +-448.
__device__ __forceinline__ uint32_t glint_f32_to_fp8(float x) {
  const uint32_t b = __float_as_uint(x);
  const uint32_t s = (b >> 24) & 0x80u;
  if ((b & 0x7fffffffu) > 0x7f800000u) return 0x7fu | s;
  const float a = fabsf(x);
  if (a >= 448.0f) return 0x7eu | s;
  if (a < 0.015625f) {                       // below 2^-6: subnormal step 2^-9
    const uint32_t m = static_cast<uint32_t>(rintf(a * 512.0f));  // 8 -> smallest normal
    return s | m;
  }
  uint32_t ab = __float_as_uint(a);
  ab += 0x7ffffu + ((ab >> 20) & 1u);        // round the 23-bit mantissa to 3 bits
  const uint32_t e = (ab >> 23) - 120u;      // rebias 127 -> 7
  const uint32_t m = (ab >> 20) & 7u;
  return s | (e << 3) | m;
}

// ---------------------------------------------------------------------------
// standard normal interval probability P(a < Z < b), accurate in both tails
// ---------------------------------------------------------------------------

__device__ __forceinline__ double glint_gauss_interval(double a, double b) {
  const double r = 0.70710678118654752440;   // 1/sqrt(2)
  double v;
  if (a >= 0.0)
    v = 0.5 * (erfc(a * r) - erfc(b * r));
  else if (b <= 0.0)
    v = 0.5 * (erfc(-b * r) - erfc(-a * r));
  else
    v = 1.0 - 0.5 * erfc(-a * r) - 0.5 * erfc(b * r);
  return v > 0.0 ? v : 0.0;
}

// ---------------------------------------------------------------------------
// cross-lane sums over aligned groups of G lanes (G a power of two <= 64);
// every lane of the group receives the group total
// ---------------------------------------------------------------------------

template <int CTRL>
__device__ __forceinline__ float glint_dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}

template <int G>
__device__ __forceinline__ float glint_group_sum(float v) {
  if constexpr (G >= 2) v += glint_dpp<0xb1>(v);    // quad_perm [1,0,3,2]
  if constexpr (G >= 4) v += glint_dpp<0x4e>(v);    // quad_perm [2,3,0,1]
  if constexpr (G >= 8) v += glint_dpp<0x141>(v);   // row_half_mirror
  if constexpr (G >= 16) v += glint_dpp<0x140>(v);  // row_mirror
  if constexpr (G >= 32) v += __shfl_xor(v, 16);
  if constexpr (G >= 64) v += __shfl_xor(v, 32);
  return v;
}

// SplitMix64 (Steele, Lea and Flood) used as a counter-based generator: the
// (counter+1)-th output of the generator seeded with `seed`, as U[0, 1).
__device__ __forceinline__ double glint_sm64_uniform(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return static_cast<double>(z >> 11) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ double glint_wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ float glint_wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Index rules of the query records.
__device__ __forceinline__ int glint_wrap(int x, int n) {
  if (static_cast<unsigned>(x) >= static_cast<unsigned>(n)) {
    x %= n;
    if (x < 0) x += n;
  }
  return x;
}

__device__ __forceinline__ int glint_clampi(int x, int lo, int hi) {
  return x < lo ? lo : (x > hi ? hi : x);
}
