// Summed-area tables, storage conversion and the constant-cost range query
// (Sec. 4.4, Eq. rangeDecom; Appendix proposition), with its gradient.
//
// Query kernel layout: a query is served by LPQ = R / RPL adjacent lanes of a
// wavefront; lane j owns ranks [j*RPL, (j+1)*RPL) and gathers its slice of
// the U and V rows with one 16-byte load each (the LPQ lanes of a query read
// one contiguous row).  The small tables (L with the per-rank scale folded
// in, CS, CT) are decoded to FP32 once per workgroup into LDS.  The rank sum
// is finished with DPP row operations inside the lane group.
#include <type_traits>

#include "common.h"

namespace {

// ---------------------------------------------------------------------------
// storage codecs for the table element types
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ float dec(T x);
template <>
__device__ __forceinline__ float dec<float>(float x) { return x; }
template <>
__device__ __forceinline__ float dec<uint16_t>(uint16_t x) { return glint_bf16_to_f32(x); }
template <>
__device__ __forceinline__ float dec<uint8_t>(uint8_t x) { return glint_fp8_to_f32(x); }

// Load RPL consecutive stored elements starting at p (16-byte aligned) and
// decode them to FP32.
template <typename FT, int RPL>
__device__ __forceinline__ void load_row(const FT* __restrict__ p, float* out) {
  constexpr int BYTES = RPL * static_cast<int>(sizeof(FT));
  static_assert(BYTES % 16 == 0, "row slice must be whole 16-byte words");
  uint4 w[BYTES / 16];
#pragma unroll
  for (int i = 0; i < BYTES / 16; ++i) w[i] = reinterpret_cast<const uint4*>(p)[i];
  const FT* e = reinterpret_cast<const FT*>(w);
#pragma unroll
  for (int i = 0; i < RPL; ++i) out[i] = dec<FT>(e[i]);
}

// Load RPL consecutive stored elements of a summed-area table row from
// global memory (aligned to the slice size) and decode them to FP32: whole
// 16-byte words where the slice allows, else one 8-, 4- or 2-byte word.
template <typename CT, int RPL>
__device__ __forceinline__ void load_cum_row(const CT* __restrict__ p, float* out) {
  constexpr int BYTES = RPL * static_cast<int>(sizeof(CT));
  if constexpr (BYTES % 16 == 0) {
    load_row<CT, RPL>(p, out);
  } else {
    static_assert(BYTES == 8 || BYTES == 4 || BYTES == 2, "row slice");
    typedef typename std::conditional<BYTES == 8, uint2,
            typename std::conditional<BYTES == 4, uint32_t, uint16_t>::type>::type W;
    const W w = *reinterpret_cast<const W*>(p);
    const CT* e = reinterpret_cast<const CT*>(&w);
#pragma unroll
    for (int i = 0; i < RPL; ++i) out[i] = dec<CT>(e[i]);
  }
}

struct Scales {
  const float* s[5];   // U, V, L, CS, CT; NULL = 1
};

// Folded per-rank scale: the product of the given per-column scales.
__device__ __forceinline__ float folded_scale(const Scales& sc, int r) {
  float c = 1.0f;
#pragma unroll
  for (int i = 0; i < 5; ++i)
    if (sc.s[i]) c *= sc.s[i][r];
  return c;
}

// Decode a stored table [rows][R] into FP32 LDS, optionally times the folded scale.
template <typename T>
__device__ void stage_table(float* __restrict__ dst, const T* __restrict__ src, int rows, int R,
                            const Scales* sc) {
  const int n = rows * R;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    float x = dec<T>(src[i]);
    if (sc) x *= folded_scale(*sc, i % R);
    dst[i] = x;
  }
}

struct QueryArgs {
  const void* U;
  const void* V;
  const void* L;
  const void* CS;
  const void* CT;
  Scales scale;
  int nu, nv, nl, N;
  int64_t nq;
  const int32_t* q;
  float* out;
};

// Row offsets of one query, resolved once by the lane that owns the query:
// element offsets of its U and V rows (global) and of its L, CS and CT rows
// (LDS).  An empty box gets equal CS offsets, so its rank terms are exact zeros.
struct alignas(16) QueryRows {
  int u, v, l, sh, sl, th, tl, pad;
};

constexpr int kQueryThreads = 512;

// RPL consecutive FP32 values from 16-byte aligned LDS.
template <int RPL>
__device__ __forceinline__ void lds_row(const float* p, float* out) {
  static_assert(RPL % 4 == 0 || RPL < 4, "row slice");
  if constexpr (RPL >= 4) {
#pragma unroll
    for (int i = 0; i < RPL / 4; ++i) {
      const float4 x = reinterpret_cast<const float4*>(p)[i];
      out[4 * i] = x.x; out[4 * i + 1] = x.y; out[4 * i + 2] = x.z; out[4 * i + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < RPL; ++i) out[i] = p[i];
  }
}

// Summed-area tables stay in LDS in BF16 when stored in BF16 (half the LDS
// bytes per gathered row; decoding is exact) and when stored in FP8 (every
// E4M3 value is exact in BF16: 3 fraction bits, exponents -9..8), otherwise
// as FP32.
template <typename CT>
struct LdsCum {
  typedef float type;
};
template <>
struct LdsCum<uint16_t> {
  typedef uint16_t type;
};
template <>
struct LdsCum<uint8_t> {
  typedef uint16_t type;
};

template <typename CT, typename LT>
__device__ void stage_cum(LT* __restrict__ dst, const CT* __restrict__ src, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    if constexpr (std::is_same<LT, uint16_t>::value && std::is_same<CT, uint16_t>::value) dst[i] = src[i];
    else if constexpr (std::is_same<LT, uint16_t>::value) dst[i] = glint_f32_to_bf16(dec<CT>(src[i]));
    else dst[i] = dec<CT>(src[i]);
  }
}

// RPL consecutive values of an LDS row (16-byte aligned for RPL*elt >= 16) as FP32.
template <typename LT, int RPL>
__device__ __forceinline__ void lds_cum_row(const LT* p, float* out) {
  if constexpr (std::is_same<LT, float>::value) {
    lds_row<RPL>(p, out);
  } else {
    static_assert(RPL % 2 == 0, "bf16 pairs");
    if constexpr (RPL >= 8) {
#pragma unroll
      for (int i = 0; i < RPL / 8; ++i) {
        const uint4 w = reinterpret_cast<const uint4*>(p)[i];
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          out[8 * i + 2 * k] = __uint_as_float(ws[k] << 16);
          out[8 * i + 2 * k + 1] = __uint_as_float(ws[k] & 0xffff0000u);
        }
      }
    } else if constexpr (RPL == 4) {
      const uint2 w = *reinterpret_cast<const uint2*>(p);
      out[0] = __uint_as_float(w.x << 16);
      out[1] = __uint_as_float(w.x & 0xffff0000u);
      out[2] = __uint_as_float(w.y << 16);
      out[3] = __uint_as_float(w.y & 0xffff0000u);
    } else {
#pragma unroll
      for (int i = 0; i < RPL; ++i) out[i] = glint_bf16_to_f32(p[i]);
    }
  }
}

// One summed-area row slice as FP32, from LDS or (GC) from global memory.
template <bool GC, typename CT, typename LT, int RPL>
__device__ __forceinline__ void cum_row(const LT* lds_tab, const CT* __restrict__ glob_tab, int off, float* out) {
  if constexpr (GC) load_cum_row<CT, RPL>(glob_tab + off, out);
  else lds_cum_row<LT, RPL>(lds_tab + off, out);
}

// Rank layout of the forward kernels: a lane's RPL ranks are RPL / CHR
// chunks of CHR ranks (CHR = one 16-byte word of the LDS summed-area rows),
// chunk c of lane j of a group of LPQ at ranks c * LPQ * CHR + j * CHR.  The
// lanes of a group then read consecutive words of a row, so one LDS
// instruction covers whole rows of several queries without bank conflicts
// (with contiguous multi-word slices every query's words fell on the same
// banks), and a group's global gathers are contiguous.  Every table uses the
// same layout; the query sums over all ranks, so which lane holds which rank
// does not matter.  Odd groups visit their chunks rotated by one (chunk c at
// position c - 1): the two 8-lane groups that share an LDS cycle at rank 64
// then read different halves of the bank space.  Sums over a lane's ranks
// add the chunk partials in the chunks' own order, so a result does not
// depend on the group that computed it.
template <typename FT, typename LT, int RPL>
constexpr int chunk_ranks_lt() {
  // BF16 factor tables over BF16 LDS rows keep one contiguous slice per lane
  // (measured faster for them; the chunked layout wins elsewhere)
  if constexpr (sizeof(FT) == 2 && sizeof(LT) == 2) return RPL;
  constexpr int w = 16 / static_cast<int>(sizeof(LT));
  return RPL < w ? RPL : w;
}

template <typename FT, typename CT, int RPL>
constexpr int chunk_ranks() {
  return chunk_ranks_lt<FT, typename LdsCum<CT>::type, RPL>();
}

template <typename T, int RPL, int CHR, int STRIDE>
__device__ __forceinline__ void load_chunks(const T* __restrict__ p, int rot, float* out) {
#pragma unroll
  for (int c = 0; c < RPL / CHR; ++c) {
    const int cc = (c + rot) & (RPL / CHR - 1);
    load_cum_row<T, CHR>(p + cc * STRIDE, out + c * CHR);
  }
}

template <int RPL, int CHR, int STRIDE>
__device__ __forceinline__ void lds_chunks(const float* p, int rot, float* out) {
#pragma unroll
  for (int c = 0; c < RPL / CHR; ++c) {
    const int cc = (c + rot) & (RPL / CHR - 1);
    lds_row<CHR>(p + cc * STRIDE, out + c * CHR);
  }
}

template <bool GC, typename CT, typename LT, int RPL, int CHR, int STRIDE>
__device__ __forceinline__ void cum_chunks(const LT* lds_tab, const CT* __restrict__ glob_tab, int off, int rot,
                                           float* out) {
#pragma unroll
  for (int c = 0; c < RPL / CHR; ++c) {
    const int cc = (c + rot) & (RPL / CHR - 1);
    cum_row<GC, CT, LT, CHR>(lds_tab, glob_tab, off + cc * STRIDE, out + c * CHR);
  }
}

// the per-chunk partials of a lane combined by a tree whose value does not
// depend on the rotation (two chunks: one commutative add; four: pairs (0,1)
// and (2,3) of the chunks' own order; more: un-rotated first)
template <int NCH>
__device__ __forceinline__ float combine_chunks(const float* p, int rot) {
  if constexpr (NCH == 1) {
    return p[0];
  } else if constexpr (NCH == 2) {
    return p[0] + p[1];
  } else if constexpr (NCH == 4) {
    // rotated by one, positions hold chunks (1, 2, 3, 0)
    const float b = rot ? p[3] : p[1], c = rot ? p[1] : p[2], d = rot ? p[2] : p[3];
    return (p[0] + b) + (c + d);
  } else {
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc += rot ? p[(c + NCH - 1) % NCH] : p[c];
    return acc;
  }
}

// sum over a lane's ranks of W ((sh - sl)(th - tl)): per-chunk partials in
// element order, combined by combine_chunks
template <int RPL, int CHR>
__device__ __forceinline__ float lane_terms(const float* W, const float* sh, const float* sl, const float* th,
                                            const float* tl, int rot) {
  constexpr int NCH = RPL / CHR;
  float p[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    float t = 0.0f;
#pragma unroll
    for (int i = 0; i < CHR; ++i) {
      const int e = c * CHR + i;
      t = fmaf(W[e], (sh[e] - sl[e]) * (th[e] - tl[e]), t);
    }
    p[c] = t;
  }
  return combine_chunks<NCH>(p, rot);
}

// lane_terms over BF16 LDS rows in 16-byte chunks (eight ranks), decoding one
// chunk of the four rows at a time: the same operations in the same order,
// with only one chunk of raw words live instead of four decoded rows
template <int RPL, int STR>
__device__ __forceinline__ float lane_terms_bf16(const float* W, const uint16_t* sh, const uint16_t* sl,
                                                 const uint16_t* th, const uint16_t* tl, int rot) {
  constexpr int CHR = 8, NCH = RPL / CHR;
  float p[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int cc = (c + rot) & (NCH - 1);
    const uint4 a = *reinterpret_cast<const uint4*>(sh + cc * STR);
    const uint4 b = *reinterpret_cast<const uint4*>(sl + cc * STR);
    const uint4 d = *reinterpret_cast<const uint4*>(th + cc * STR);
    const uint4 f = *reinterpret_cast<const uint4*>(tl + cc * STR);
    const uint32_t A[4] = {a.x, a.y, a.z, a.w}, B[4] = {b.x, b.y, b.z, b.w};
    const uint32_t D[4] = {d.x, d.y, d.z, d.w}, F[4] = {f.x, f.y, f.z, f.w};
    float t = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = c * CHR + 2 * k;
      t = fmaf(W[e], (__uint_as_float(A[k] << 16) - __uint_as_float(B[k] << 16)) *
                         (__uint_as_float(D[k] << 16) - __uint_as_float(F[k] << 16)), t);
      t = fmaf(W[e + 1], (__uint_as_float(A[k] & 0xffff0000u) - __uint_as_float(B[k] & 0xffff0000u)) *
                             (__uint_as_float(D[k] & 0xffff0000u) - __uint_as_float(F[k] & 0xffff0000u)), t);
    }
    p[c] = t;
  }
  return combine_chunks<NCH>(p, rot);
}

// A resolved record of the flat query, 16 bytes: u | l << 26, v, and the
// two tables' row pairs (hi | lo << 16): in LDS as byte offsets / 16, with
// GC as row indices.
struct alignas(16) PackedRows {
  uint32_t ul, v, a, b;
};

// The four summed-area row slices of a resolved record (CS hi, CS lo, CT hi,
// CT lo; for an odd group the two tables come swapped, see k_query).
template <bool GC, typename CT, typename LT, int RPL, int CHR, int STR, int R>
__device__ __forceinline__ void record_rows(const PackedRows& r, const unsigned char* cum_lane,
                                            const LT* CSs, const LT* CTs, const CT* __restrict__ CSg,
                                            const CT* __restrict__ CTg, int r0, float* sh, float* sl,
                                            float* th, float* tl) {
  if constexpr (GC) {
    cum_chunks<true, CT, LT, RPL, CHR, STR>(CSs, CSg, static_cast<int>(r.a & 0xffffu) * R + r0, 0, sh);
    cum_chunks<true, CT, LT, RPL, CHR, STR>(CSs, CSg, static_cast<int>(r.a >> 16) * R + r0, 0, sl);
    cum_chunks<true, CT, LT, RPL, CHR, STR>(CTs, CTg, static_cast<int>(r.b & 0xffffu) * R + r0, 0, th);
    cum_chunks<true, CT, LT, RPL, CHR, STR>(CTs, CTg, static_cast<int>(r.b >> 16) * R + r0, 0, tl);
  } else {
    const LT* ah = reinterpret_cast<const LT*>(cum_lane + ((r.a & 0xffffu) << 4));
    const LT* al = reinterpret_cast<const LT*>(cum_lane + ((r.a >> 16) << 4));
    const LT* bh = reinterpret_cast<const LT*>(cum_lane + ((r.b & 0xffffu) << 4));
    const LT* bl = reinterpret_cast<const LT*>(cum_lane + ((r.b >> 16) << 4));
    cum_chunks<false, CT, LT, RPL, CHR, STR>(ah, CSg, 0, 0, sh);
    cum_chunks<false, CT, LT, RPL, CHR, STR>(al, CSg, 0, 0, sl);
    cum_chunks<false, CT, LT, RPL, CHR, STR>(bh, CTg, 0, 0, th);
    cum_chunks<false, CT, LT, RPL, CHR, STR>(bl, CTg, 0, 0, tl);
  }
}


// LDS layout of the flat query: L (FP32) at 0, CS at a 256-byte boundary,
// CT half a bank width (128 bytes) past the next 256-byte boundary, then
// the record slots.  With GC the summed-area tables stay in global memory.
struct QueryLds {
  size_t cs, ct, rows, total;
};

__host__ __device__ inline QueryLds query_lds(int nl, int N, int R, size_t lt_bytes, bool gc, size_t slot_bytes) {
  QueryLds o;
  const size_t l_bytes = sizeof(float) * static_cast<size_t>(nl) * R;
  const size_t table = lt_bytes * static_cast<size_t>(N + 1) * R;
  if (gc) {
    o.cs = o.ct = 0;
    o.rows = glint_round_up(l_bytes, 16);
  } else {
    o.cs = glint_round_up(l_bytes, 256);
    o.ct = glint_round_up(o.cs + table, 256) + 128;
    o.rows = glint_round_up(o.ct + table, 16);
  }
  o.total = o.rows + slot_bytes;
  return o;
}

// GC: the summed-area tables are too large for LDS and are read from global
// memory (L2-resident); L stays in LDS.  LT is the element type of the LDS
// copies of the summed-area tables (FP32, or BF16 kept as stored).
//
// LDS bank spreading: the lane groups of a wave read their rows' chunks in
// the same order, and the rows of one table all start on the same bank, so
// odd groups read the CT rows where even groups read the CS rows (CT sits
// half a bank width off CS).  The term of a rank is W (dS dT), symmetric in
// the two tables, so the swap leaves every value unchanged.
// NT threads per block; at 1024 the compiler is held to 64 VGPRs (eight
// waves per SIMD), so two blocks of 16 waves share a CU with one copy of
// the tables each.

template <typename FT, typename CT, typename LT, int R, int RPL, bool GC, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT == 1024 ? 8 : 1))) void k_query(QueryArgs a) {
  constexpr int LPQ = R / RPL;           // lanes per query
  static_assert(LPQ >= 1 && LPQ <= 64, "lanes per query");
  static_assert(std::is_same<LT, float>::value || std::is_same<LT, CT>::value ||
                    (std::is_same<LT, uint16_t>::value && std::is_same<CT, uint8_t>::value),
                "LDS copy type");
  constexpr int kSlots = 64 + 64 / LPQ;
  extern __shared__ __align__(16) float lds[];
  unsigned char* lds_b = reinterpret_cast<unsigned char*>(lds);
  const QueryLds lay = query_lds(a.nl, a.N, R, sizeof(LT), GC, 0);
  float* Ls = lds;
  LT* CSs = reinterpret_cast<LT*>(lds_b + lay.cs);
  LT* CTs = reinterpret_cast<LT*>(lds_b + lay.ct);
  PackedRows* rows = reinterpret_cast<PackedRows*>(lds_b + lay.rows);
  const CT* CSg = static_cast<const CT*>(a.CS);
  const CT* CTg = static_cast<const CT*>(a.CT);
  stage_table<FT>(Ls, static_cast<const FT*>(a.L), a.nl, R, &a.scale);
  if constexpr (!GC) {
    stage_cum<CT, LT>(CSs, CSg, (a.N + 1) * R);
    stage_cum<CT, LT>(CTs, CTg, (a.N + 1) * R);
  }
  __syncthreads();

  const FT* __restrict__ U = static_cast<const FT*>(a.U);
  const FT* __restrict__ V = static_cast<const FT*>(a.V);
  const int lane = threadIdx.x & 63;
  const int g = lane / LPQ;
  const int j = lane % LPQ;
  constexpr int CHR = chunk_ranks_lt<FT, LT, RPL>();
  constexpr int STR = LPQ * CHR;
  const int r0 = j * CHR;
  // record slots: query g*LPQ + jj sits at g*(LPQ+1) + jj, so the groups' slots
  // do not share LDS banks when read back
  PackedRows* wrows = rows + (threadIdx.x >> 6) * kSlots;
  const int my_slot = lane + lane / LPQ;
  // the lane's own columns of the LDS summed-area rows (record offsets are bytes from lds)
  const unsigned char* cum_lane = lds_b + r0 * sizeof(LT);
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < a.nq; base += nwaves * 64) {
    // phase 1: lane i resolves query base + i (all seven loads issued first)
    {
      const int64_t qi = base + lane;
      const int64_t qc = qi < a.nq ? qi : a.nq - 1;
      const int32_t* rec = a.q + qc * 7;
      // records and results stream through once: non-temporal loads and
      // stores keep them from evicting the U and V rows gathered from the
      // L2 (rank-128 headline batch: fetched bytes 1.136x -> 1.037x the
      // records' bytes).  The grouped query keeps plain loads and stores:
      // non-temporal box loads and result stores there raised its fetched
      // bytes 2.3x.
      int f[7];
#pragma unroll
      for (int i = 0; i < 7; ++i) f[i] = __builtin_nontemporal_load(rec + i);
      const int u = glint_wrap(f[0], a.nu);
      const int v = glint_wrap(f[1], a.nv);
      const int l = glint_clampi(f[2], 0, a.nl - 1);
      const int slo = glint_clampi(f[3], 0, a.N), shi = glint_clampi(f[4], 0, a.N);
      const int tlo = glint_clampi(f[5], 0, a.N), thi = glint_clampi(f[6], 0, a.N);
      const bool empty = !(slo < shi && tlo < thi);
      const int s_hi = empty ? slo : shi;
      PackedRows r;
      r.ul = static_cast<uint32_t>(u) | static_cast<uint32_t>(l) << 26;
      r.v = static_cast<uint32_t>(v);
      if constexpr (GC) {
        // row indices into the global tables
        r.a = static_cast<uint32_t>(s_hi) | static_cast<uint32_t>(slo) << 16;
        r.b = static_cast<uint32_t>(thi) | static_cast<uint32_t>(tlo) << 16;
      } else {
        // byte offsets from lds / 16; the group that serves this query
        // (lane / LPQ) takes CT first when odd
        constexpr uint32_t RB = static_cast<uint32_t>(sizeof(LT)) * R;   // bytes per row
        const uint32_t cs = static_cast<uint32_t>(lay.cs), ct = static_cast<uint32_t>(lay.ct);
        const uint32_t sp = ((cs + s_hi * RB) >> 4) | ((cs + slo * RB) >> 4) << 16;
        const uint32_t tp = ((ct + thi * RB) >> 4) | ((ct + tlo * RB) >> 4) << 16;
        const bool odd = (lane / LPQ) & 1;
        r.a = odd ? tp : sp;
        r.b = odd ? sp : tp;
      }
      wrows[my_slot] = r;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // phase 2: group g serves queries g*LPQ .. g*LPQ + LPQ - 1; lane j keeps query
    // g*LPQ + j.  The footprint product W = U*V*L is reused while consecutive
    // queries share (u, v, l) (several angular boxes of one shading point).
    float res = 0.0f;
    uint32_t pul = ~0u, pv = ~0u;
    float W[RPL];
#pragma unroll 2
    for (int jj = 0; jj < LPQ; ++jj) {
      const PackedRows r = wrows[g * (LPQ + 1) + jj];
      if (r.ul != pul || r.v != pv) {
        float uu[RPL], vv[RPL], lr[RPL];
        load_chunks<FT, RPL, CHR, STR>(U + static_cast<int64_t>(r.ul & 0x3ffffffu) * R + r0, 0, uu);
        load_chunks<FT, RPL, CHR, STR>(V + static_cast<int64_t>(r.v) * R + r0, 0, vv);
        lds_chunks<RPL, CHR, STR>(Ls + (r.ul >> 26) * R + r0, 0, lr);
#pragma unroll
        for (int e = 0; e < RPL; ++e) W[e] = uu[e] * vv[e] * lr[e];
        pul = r.ul; pv = r.v;
      }
      float sh[RPL], sl[RPL], th[RPL], tl[RPL];
      record_rows<GC, CT, LT, RPL, CHR, STR, R>(r, cum_lane, CSs, CTs, CSg, CTg, r0, sh, sl, th, tl);
      float acc = lane_terms<RPL, CHR>(W, sh, sl, th, tl, 0);
      acc = glint_group_sum<LPQ>(acc);
      res = (j == jj) ? acc : res;
    }
    __builtin_amdgcn_wave_barrier();
    const int64_t qo = base + g * LPQ + j;
    if (qo < a.nq) __builtin_nontemporal_store(res, a.out + qo);
  }
}

struct GroupedArgs {
  const void* U;
  const void* V;
  const void* L;
  const void* CS;
  const void* CT;
  Scales scale;
  int nu, nv, nl, N, K;
  int64_t npts;
  const int32_t* uvl;
  const int32_t* boxes;
  float* out;
};

// Grouped query: lane i of a wave resolves shading point base + i to row
// offsets; lane group g then takes points g*LPQ .. g*LPQ + LPQ - 1 one by one,
// forms W = U*V*L once per point and walks its K boxes, only the summed-area
// rows changing per box.  Lane j keeps the result of box b with b % LPQ == j,
// so LPQ consecutive results leave as one contiguous store.
template <typename FT, typename CT, int R, int RPL, bool GC, int NT>
__global__ __launch_bounds__(NT) void k_query_grouped(GroupedArgs a) {
  constexpr int LPQ = R / RPL;
  typedef typename LdsCum<CT>::type LT;
  extern __shared__ __align__(16) float lds[];
  float* Ls = lds;
  LT* CSs = reinterpret_cast<LT*>(Ls + a.nl * R);
  LT* CTs = CSs + (a.N + 1) * R;
  const size_t cum_bytes = GC ? 0 : 2 * sizeof(LT) * (a.N + 1) * R;
  int4* pts = reinterpret_cast<int4*>(
      reinterpret_cast<unsigned char*>(lds) + glint_round_up(sizeof(float) * a.nl * R + cum_bytes, 16));
  const CT* CSg = static_cast<const CT*>(a.CS);
  const CT* CTg = static_cast<const CT*>(a.CT);
  stage_table<FT>(Ls, static_cast<const FT*>(a.L), a.nl, R, &a.scale);
  if constexpr (!GC) {
    stage_cum<CT, LT>(CSs, CSg, (a.N + 1) * R);
    stage_cum<CT, LT>(CTs, CTg, (a.N + 1) * R);
  }
  __syncthreads();

  const FT* __restrict__ U = static_cast<const FT*>(a.U);
  const FT* __restrict__ V = static_cast<const FT*>(a.V);
  const int lane = threadIdx.x & 63;
  const int g = lane / LPQ;
  const int j = lane % LPQ;
  constexpr int CHR = chunk_ranks<FT, CT, RPL>();
  constexpr int STR = LPQ * CHR;
  const int r0 = j * CHR;
  const int rot = RPL / CHR > 1 ? (g & 1) : 0;
  const int K = a.K;
  int4* wpts = pts + (threadIdx.x >> 6) * 64;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < a.npts; base += nwaves * 64) {
    {
      const int64_t pi = base + lane;
      const int64_t pc = pi < a.npts ? pi : a.npts - 1;
      const int32_t* rec = a.uvl + pc * 3;
      const int f0 = rec[0], f1 = rec[1], f2 = rec[2];
      wpts[lane] = make_int4(glint_wrap(f0, a.nu) * R, glint_wrap(f1, a.nv) * R,
                             glint_clampi(f2, 0, a.nl - 1) * R, 0);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    for (int jj = 0; jj < LPQ; ++jj) {
      const int64_t pi = base + g * LPQ + jj;
      if (pi >= a.npts) break;                // group-uniform: no cross-group operations follow
      const int4 pr = wpts[g * LPQ + jj];
      float W[RPL];
      {
        float uu[RPL], vv[RPL], lr[RPL];
        load_chunks<FT, RPL, CHR, STR>(U + pr.x + r0, rot, uu);
        load_chunks<FT, RPL, CHR, STR>(V + pr.y + r0, rot, vv);
        lds_chunks<RPL, CHR, STR>(Ls + pr.z + r0, rot, lr);
#pragma unroll
        for (int e = 0; e < RPL; ++e) W[e] = uu[e] * vv[e] * lr[e];
      }
      const int4* bx = reinterpret_cast<const int4*>(a.boxes) + pi * K;
      float* out = a.out + pi * K;
      float res = 0.0f;
      // each box record is loaded one box ahead, before the previous results' store
      int4 nbox = K > 0 ? bx[0] : make_int4(0, 0, 0, 0);
      for (int b = 0; b < K; ++b) {
        const int4 box = nbox;
        if (b + 1 < K) nbox = bx[b + 1];
        const int slo = glint_clampi(box.x, 0, a.N), shi0 = glint_clampi(box.y, 0, a.N);
        const int tlo = glint_clampi(box.z, 0, a.N), thi = glint_clampi(box.w, 0, a.N);
        const int shi = (slo < shi0 && tlo < thi) ? shi0 : slo;     // empty box: exact zeros
        float acc;
        if constexpr (!GC && std::is_same<LT, uint16_t>::value && CHR == 8) {
          acc = lane_terms_bf16<RPL, STR>(W, CSs + shi * R + r0, CSs + slo * R + r0, CTs + thi * R + r0,
                                          CTs + tlo * R + r0, rot);
        } else {
          float sh[RPL], sl[RPL], th[RPL], tl[RPL];
          cum_chunks<GC, CT, LT, RPL, CHR, STR>(CSs, CSg, shi * R + r0, rot, sh);
          cum_chunks<GC, CT, LT, RPL, CHR, STR>(CSs, CSg, slo * R + r0, rot, sl);
          cum_chunks<GC, CT, LT, RPL, CHR, STR>(CTs, CTg, thi * R + r0, rot, th);
          cum_chunks<GC, CT, LT, RPL, CHR, STR>(CTs, CTg, tlo * R + r0, rot, tl);
          acc = lane_terms<RPL, CHR>(W, sh, sl, th, tl, rot);
        }
        acc = glint_group_sum<LPQ>(acc);
        const int bj = b % LPQ;
        res = (j == bj) ? acc : res;
        if (bj == LPQ - 1 || b == K - 1) {
          if (j <= bj) out[b - bj + j] = res;
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Off-grid footprints (Sec. 4.1, Sec. 4.3): the trilinear blend of the range
// queries of the eight precomputed footprints around a continuous centre
// (x, y) and level lam.  The reconstruction is multilinear in the U, V and L
// rows, so the blend equals one query with linearly interpolated rows: two
// U, two V (global) and two L (LDS) rows per record instead of one each.
// Coordinates are in index units; a non-finite coordinate counts as 0,
// |x|, |y| are clamped to 2^24, x and y wrap, lam clamps to [0, nl - 1].
struct TriArgs {
  const void* U;
  const void* V;
  const void* L;
  const void* CS;
  const void* CT;
  Scales scale;
  int nu, nv, nl, N;
  int64_t nq;
  const float* xyl;
  const int32_t* boxes;
  float* out;
};

// A resolved trilinear record, 32 bytes: u0 | l0 << 26, v0, the two tables'
// row pairs (hi | lo << 16, row indices) and the three blend weights; the
// upper corners u0 + 1, v0 + 1 (wrapped) and l0 + 1 (clamped) are derived
// when the footprint changes.
struct alignas(16) TriRows {
  uint32_t ul, v, s, t;
  float wx, wy, wl, pad;
};

constexpr float kCoordLimit = 16777216.0f;

__device__ __forceinline__ float finite_or_zero(float x) { return __builtin_isfinite(x) ? x : 0.0f; }

template <typename FT, typename CT, int R, int RPL, bool GC>
__global__ __launch_bounds__(kQueryThreads) void k_query_trilinear(TriArgs a) {
  constexpr int LPQ = R / RPL;
  typedef typename LdsCum<CT>::type LT;
  extern __shared__ __align__(16) float lds[];
  float* Ls = lds;
  LT* CSs = reinterpret_cast<LT*>(Ls + a.nl * R);
  LT* CTs = CSs + (a.N + 1) * R;
  const size_t cum_bytes = GC ? 0 : 2 * sizeof(LT) * (a.N + 1) * R;
  TriRows* rows = reinterpret_cast<TriRows*>(
      reinterpret_cast<unsigned char*>(lds) + glint_round_up(sizeof(float) * a.nl * R + cum_bytes, 16));
  const CT* CSg = static_cast<const CT*>(a.CS);
  const CT* CTg = static_cast<const CT*>(a.CT);
  stage_table<FT>(Ls, static_cast<const FT*>(a.L), a.nl, R, &a.scale);
  if constexpr (!GC) {
    stage_cum<CT, LT>(CSs, CSg, (a.N + 1) * R);
    stage_cum<CT, LT>(CTs, CTg, (a.N + 1) * R);
  }
  __syncthreads();

  const FT* __restrict__ U = static_cast<const FT*>(a.U);
  const FT* __restrict__ V = static_cast<const FT*>(a.V);
  const int lane = threadIdx.x & 63;
  const int g = lane / LPQ;
  const int j = lane % LPQ;
  constexpr int CHR = chunk_ranks<FT, CT, RPL>();
  constexpr int STR = LPQ * CHR;
  const int r0 = j * CHR;
  const int rot = RPL / CHR > 1 ? (g & 1) : 0;
  constexpr int kSlots = 64 + 64 / LPQ;
  TriRows* wrows = rows + (threadIdx.x >> 6) * kSlots;
  const int my_slot = lane + lane / LPQ;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < a.nq; base += nwaves * 64) {
    {
      const int64_t qi = base + lane;
      const int64_t qc = qi < a.nq ? qi : a.nq - 1;
      const float* c = a.xyl + qc * 3;
      const int32_t* bx = a.boxes + qc * 4;
      float x = finite_or_zero(c[0]), y = finite_or_zero(c[1]), lam = finite_or_zero(c[2]);
      const int b0 = bx[0], b1 = bx[1], b2 = bx[2], b3 = bx[3];
      x = fminf(fmaxf(x, -kCoordLimit), kCoordLimit);
      y = fminf(fmaxf(y, -kCoordLimit), kCoordLimit);
      lam = fminf(fmaxf(lam, 0.0f), static_cast<float>(a.nl - 1));
      const float fx = floorf(x), fy = floorf(y), fl = floorf(lam);
      const int ix = static_cast<int>(fx), iy = static_cast<int>(fy), il = static_cast<int>(fl);
      const int slo = glint_clampi(b0, 0, a.N), shi = glint_clampi(b1, 0, a.N);
      const int tlo = glint_clampi(b2, 0, a.N), thi = glint_clampi(b3, 0, a.N);
      const bool empty = !(slo < shi && tlo < thi);
      TriRows r;
      r.ul = static_cast<uint32_t>(glint_wrap(ix, a.nu)) | static_cast<uint32_t>(il) << 26;
      r.v = static_cast<uint32_t>(glint_wrap(iy, a.nv));
      r.s = static_cast<uint32_t>(empty ? slo : shi) | static_cast<uint32_t>(slo) << 16;
      r.t = static_cast<uint32_t>(thi) | static_cast<uint32_t>(tlo) << 16;
      r.wx = x - fx;
      r.wy = y - fy;
      r.wl = lam - fl;
      r.pad = 0.0f;
      wrows[my_slot] = r;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    float res = 0.0f;
    // the interpolated footprint product is reused while consecutive records
    // share the centre and level (several boxes of one shading point)
    uint32_t pul = ~0u, pv = ~0u;
    float pwx = -1.0f, pwy = -1.0f, pwl = -1.0f;
    float W[RPL];
    for (int jj = 0; jj < LPQ; ++jj) {
      const TriRows r = wrows[g * (LPQ + 1) + jj];
      if (r.ul != pul || r.v != pv || r.wx != pwx || r.wy != pwy || r.wl != pwl) {
        const int u0 = static_cast<int>(r.ul & 0x3ffffffu), l0 = static_cast<int>(r.ul >> 26);
        const int v0 = static_cast<int>(r.v);
        const int u1 = u0 + 1 == a.nu ? 0 : u0 + 1, v1 = v0 + 1 == a.nv ? 0 : v0 + 1;
        const int l1 = min(l0 + 1, a.nl - 1);
        float ua[RPL], ub[RPL], va[RPL], vb[RPL], la[RPL], lb[RPL];
        load_chunks<FT, RPL, CHR, STR>(U + static_cast<int64_t>(u0) * R + r0, rot, ua);
        load_chunks<FT, RPL, CHR, STR>(U + static_cast<int64_t>(u1) * R + r0, rot, ub);
        load_chunks<FT, RPL, CHR, STR>(V + static_cast<int64_t>(v0) * R + r0, rot, va);
        load_chunks<FT, RPL, CHR, STR>(V + static_cast<int64_t>(v1) * R + r0, rot, vb);
        lds_chunks<RPL, CHR, STR>(Ls + l0 * R + r0, rot, la);
        lds_chunks<RPL, CHR, STR>(Ls + l1 * R + r0, rot, lb);
#pragma unroll
        for (int e = 0; e < RPL; ++e)
          W[e] = (ua[e] + r.wx * (ub[e] - ua[e])) * (va[e] + r.wy * (vb[e] - va[e])) *
                 (la[e] + r.wl * (lb[e] - la[e]));
        pul = r.ul; pv = r.v;
        pwx = r.wx; pwy = r.wy; pwl = r.wl;
      }
      float sh[RPL], sl[RPL], th[RPL], tl[RPL];
      cum_chunks<GC, CT, LT, RPL, CHR, STR>(CSs, CSg, static_cast<int>(r.s & 0xffffu) * R + r0, rot, sh);
      cum_chunks<GC, CT, LT, RPL, CHR, STR>(CSs, CSg, static_cast<int>(r.s >> 16) * R + r0, rot, sl);
      cum_chunks<GC, CT, LT, RPL, CHR, STR>(CTs, CTg, static_cast<int>(r.t & 0xffffu) * R + r0, rot, th);
      cum_chunks<GC, CT, LT, RPL, CHR, STR>(CTs, CTg, static_cast<int>(r.t >> 16) * R + r0, rot, tl);
      float acc = lane_terms<RPL, CHR>(W, sh, sl, th, tl, rot);
      acc = glint_group_sum<LPQ>(acc);
      res = (j == jj) ? acc : res;
    }
    __builtin_amdgcn_wave_barrier();
    const int64_t qo = base + g * LPQ + j;
    if (qo < a.nq) a.out[qo] = res;
  }
}

// Hierarchical importance sampling of the NDF image of a footprint (Sec.
// 5.2): the image is split into four quads whose masses come from range
// queries, one is drawn in proportion to its mass (negative masses count as
// zero), and the split repeats inside it for log2(N) levels; the sample is
// then placed uniformly inside the final bin.  One lane group per sample:
// W = U V L once, the current bounds' summed-area rows carried in registers,
// two new rows (the midpoints) and one four-way group reduction per level.
// The choice is taken by the group's first lane and broadcast.  A sample
// whose quads hold no positive mass fails: bin (-1, -1), pdf 0, h = (0, 0).
struct SampleArgs {
  const void* U;
  const void* V;
  const void* L;
  const void* CS;
  const void* CT;
  Scales scale;
  int nu, nv, nl, N, levels;
  int64_t n;
  const int32_t* uvl;
  const float* rnd;     // [n][levels + 2]
  float* h;             // [n][2]
  float* pdf;           // [n]
  int32_t* bins;        // [n][2]
};

template <typename FT, typename CT, int R, int RPL, bool GC>
__global__ __launch_bounds__(kQueryThreads) void k_sample(SampleArgs a) {
  constexpr int LPQ = R / RPL;
  typedef typename LdsCum<CT>::type LT;
  extern __shared__ __align__(16) float lds[];
  float* Ls = lds;
  LT* CSs = reinterpret_cast<LT*>(Ls + a.nl * R);
  LT* CTs = CSs + (a.N + 1) * R;
  const size_t cum_bytes = GC ? 0 : 2 * sizeof(LT) * (a.N + 1) * R;
  int4* pts = reinterpret_cast<int4*>(
      reinterpret_cast<unsigned char*>(lds) + glint_round_up(sizeof(float) * a.nl * R + cum_bytes, 16));
  const CT* CSg = static_cast<const CT*>(a.CS);
  const CT* CTg = static_cast<const CT*>(a.CT);
  stage_table<FT>(Ls, static_cast<const FT*>(a.L), a.nl, R, &a.scale);
  if constexpr (!GC) {
    stage_cum<CT, LT>(CSs, CSg, (a.N + 1) * R);
    stage_cum<CT, LT>(CTs, CTg, (a.N + 1) * R);
  }
  __syncthreads();

  const FT* __restrict__ U = static_cast<const FT*>(a.U);
  const FT* __restrict__ V = static_cast<const FT*>(a.V);
  const int lane = threadIdx.x & 63;
  const int g = lane / LPQ;
  const int j = lane % LPQ;
  constexpr int CHR = chunk_ranks<FT, CT, RPL>();
  constexpr int STR = LPQ * CHR;
  const int r0 = j * CHR;
  const int rot = RPL / CHR > 1 ? (g & 1) : 0;
  const int nr = a.levels + 2;
  const float w = 2.0f / static_cast<float>(a.N);
  int4* wpts = pts + (threadIdx.x >> 6) * 64;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < a.n; base += nwaves * 64) {
    {
      const int64_t pi = base + lane;
      const int64_t pc = pi < a.n ? pi : a.n - 1;
      const int32_t* rec = a.uvl + pc * 3;
      const int f0 = rec[0], f1 = rec[1], f2 = rec[2];
      wpts[lane] = make_int4(glint_wrap(f0, a.nu) * R, glint_wrap(f1, a.nv) * R,
                             glint_clampi(f2, 0, a.nl - 1) * R, 0);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    float hs = 0.0f, ht = 0.0f, pd = 0.0f;
    int bs = -1, bt = -1;
    for (int jj = 0; jj < LPQ; ++jj) {
      const int64_t pi = base + g * LPQ + jj;
      if (pi >= a.n) break;                 // group-uniform
      const int4 pr = wpts[g * LPQ + jj];
      float W[RPL];
      {
        float uu[RPL], vv[RPL], lr[RPL];
        load_chunks<FT, RPL, CHR, STR>(U + pr.x + r0, rot, uu);
        load_chunks<FT, RPL, CHR, STR>(V + pr.y + r0, rot, vv);
        lds_chunks<RPL, CHR, STR>(Ls + pr.z + r0, rot, lr);
#pragma unroll
        for (int e = 0; e < RPL; ++e) W[e] = uu[e] * vv[e] * lr[e];
      }
      const float* rn = a.rnd + pi * nr;
      int s0 = 0, s1 = a.N, t0 = 0, t1 = a.N;
      float cs0[RPL], cs1[RPL], ct0[RPL], ct1[RPL];
      cum_chunks<GC, CT, LT, RPL, CHR, STR>(CSs, CSg, r0, rot, cs0);
      cum_chunks<GC, CT, LT, RPL, CHR, STR>(CSs, CSg, a.N * R + r0, rot, cs1);
      cum_chunks<GC, CT, LT, RPL, CHR, STR>(CTs, CTg, r0, rot, ct0);
      cum_chunks<GC, CT, LT, RPL, CHR, STR>(CTs, CTg, a.N * R + r0, rot, ct1);
      float prob = 1.0f;
      bool ok = true;
      for (int k = 0; k < a.levels; ++k) {
        const int sm = (s0 + s1) >> 1, tm = (t0 + t1) >> 1;
        float csm[RPL], ctm[RPL];
        cum_chunks<GC, CT, LT, RPL, CHR, STR>(CSs, CSg, sm * R + r0, rot, csm);
        cum_chunks<GC, CT, LT, RPL, CHR, STR>(CTs, CTg, tm * R + r0, rot, ctm);
        float q00 = 0.0f, q01 = 0.0f, q10 = 0.0f, q11 = 0.0f;
#pragma unroll
        for (int e = 0; e < RPL; ++e) {
          const float sl = csm[e] - cs0[e], sh = cs1[e] - csm[e];
          const float tl = ctm[e] - ct0[e], th = ct1[e] - ctm[e];
          const float ws = W[e] * sl, wh = W[e] * sh;
          q00 += ws * tl;
          q01 += ws * th;
          q10 += wh * tl;
          q11 += wh * th;
        }
        q00 = glint_group_sum<LPQ>(q00);
        q01 = glint_group_sum<LPQ>(q01);
        q10 = glint_group_sum<LPQ>(q10);
        q11 = glint_group_sum<LPQ>(q11);
        const float m0 = fmaxf(q00, 0.0f), m1 = fmaxf(q01, 0.0f), m2 = fmaxf(q10, 0.0f), m3 = fmaxf(q11, 0.0f);
        const float total = ((m0 + m1) + m2) + m3;
        int pick = -1;
        if (total > 0.0f) {
          const float target = rn[k] * total;
          float run = m0;
          pick = 3;
          if (target < run) pick = 0;
          else if (target < (run += m1)) pick = 1;
          else if (target < (run += m2)) pick = 2;
          // never an empty quad (the target can meet the top of the range by rounding)
          if (pick == 3 && !(m3 > 0.0f)) pick = m2 > 0.0f ? 2 : (m1 > 0.0f ? 1 : 0);
        }
        pick = __shfl(pick, g * LPQ);      // one decision per group
        if (pick < 0) {
          ok = false;
          break;
        }
        const float mp = pick == 0 ? m0 : (pick == 1 ? m1 : (pick == 2 ? m2 : m3));
        prob *= __shfl(mp / total, g * LPQ);
        if (pick >= 2) {
          s0 = sm;
#pragma unroll
          for (int e = 0; e < RPL; ++e) cs0[e] = csm[e];
        } else {
          s1 = sm;
#pragma unroll
          for (int e = 0; e < RPL; ++e) cs1[e] = csm[e];
        }
        if (pick & 1) {
          t0 = tm;
#pragma unroll
          for (int e = 0; e < RPL; ++e) ct0[e] = ctm[e];
        } else {
          t1 = tm;
#pragma unroll
          for (int e = 0; e < RPL; ++e) ct1[e] = ctm[e];
        }
      }
      if (j == jj) {
        if (ok) {
          bs = s0;
          bt = t0;
          hs = -1.0f + (static_cast<float>(s0) + rn[a.levels]) * w;
          ht = -1.0f + (static_cast<float>(t0) + rn[a.levels + 1]) * w;
          pd = prob / (w * w);
        } else {
          bs = bt = -1;
          hs = ht = pd = 0.0f;
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    const int64_t qo = base + g * LPQ + j;
    if (qo < a.n) {
      a.h[2 * qo] = hs;
      a.h[2 * qo + 1] = ht;
      a.pdf[qo] = pd;
      a.bins[2 * qo] = bs;
      a.bins[2 * qo + 1] = bt;
    }
  }
}

// Backward.  Phase 1 (one lane per query, as in the forward) resolves the
// record and its upstream gradient (0 for empty boxes and padding, so those
// contribute exact zeros).  Phase 2: lane group g walks its LPQ consecutive
// queries; lane j owns ranks [j*RPL, (j+1)*RPL).  dU, dV, dL accumulate in
// registers while (u, v, l) repeat and are flushed with one atomic per rank
// when they change (consecutive boxes of one shading point share them); the
// summed-area-table gradients go to LDS accumulators (few rows, heavily
// shared) and are flushed once per block.
template <typename FT, typename CT, int R, int RPL>
__global__ __launch_bounds__(kQueryThreads) void k_query_backward(QueryArgs a, const float* __restrict__ gout,
                                                                  float* __restrict__ dU,
                                                                  float* __restrict__ dV,
                                                                  float* __restrict__ dL,
                                                                  float* __restrict__ dCS,
                                                                  float* __restrict__ dCT) {
  constexpr int LPQ = R / RPL;
  extern __shared__ __align__(16) float lds[];
  const int nl = a.nl, N1 = a.N + 1;
  float* Ls = lds;                  // decoded L (no scale)
  float* CSs = Ls + nl * R;
  float* CTs = CSs + N1 * R;
  float* sc = CTs + N1 * R;         // [R] folded scale
  float* gL = sc + R;               // [nl][R]
  float* gCS = gL + nl * R;         // [N1][R]
  float* gCT = gCS + N1 * R;        // [N1][R]
  QueryRows* rows = reinterpret_cast<QueryRows*>(gCT + N1 * R);
  stage_table<FT>(Ls, static_cast<const FT*>(a.L), nl, R, nullptr);
  stage_table<CT>(CSs, static_cast<const CT*>(a.CS), N1, R, nullptr);
  stage_table<CT>(CTs, static_cast<const CT*>(a.CT), N1, R, nullptr);
  for (int i = threadIdx.x; i < R; i += blockDim.x) sc[i] = folded_scale(a.scale, i);
  for (int i = threadIdx.x; i < (nl + 2 * N1) * R; i += blockDim.x) gL[i] = 0.0f;
  __syncthreads();

  const FT* __restrict__ U = static_cast<const FT*>(a.U);
  const FT* __restrict__ V = static_cast<const FT*>(a.V);
  const int lane = threadIdx.x & 63;
  const int g = lane / LPQ;
  const int j = lane % LPQ;
  const int r0 = j * RPL;
  float scr[RPL];
#pragma unroll
  for (int e = 0; e < RPL; ++e) scr[e] = sc[r0 + e];
  QueryRows* wrows = rows + (threadIdx.x >> 6) * 64;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  // running (u, v, l) of this group and its register accumulators
  int cu = -1, cv = -1, cl = -1;
  float aU[RPL], aV[RPL], aL[RPL];
#pragma unroll
  for (int e = 0; e < RPL; ++e) aU[e] = aV[e] = aL[e] = 0.0f;
  // The LDS gradient rows are swizzled: lane j's rank r0 + e sits at e*LPQ + j,
  // so each atomic instruction of a lane group hits consecutive words (no bank
  // conflicts); the rows are unswizzled when the block adds them to global memory.
  auto flush = [&]() {
    if (cu >= 0) {
#pragma unroll
      for (int e = 0; e < RPL; ++e) {
        if (aU[e] != 0.0f) atomicAdd(&dU[cu + r0 + e], aU[e]);
        if (aV[e] != 0.0f) atomicAdd(&dV[cv + r0 + e], aV[e]);
        if (aL[e] != 0.0f) atomicAdd(&gL[cl + e * LPQ + j], aL[e]);
        aU[e] = aV[e] = aL[e] = 0.0f;
      }
    }
  };
  for (int64_t base = wave * 64; base < a.nq; base += nwaves * 64) {
    {
      const int64_t qi = base + lane;
      const int64_t qc = qi < a.nq ? qi : a.nq - 1;
      const int32_t* rec = a.q + qc * 7;
      int f[7];
#pragma unroll
      for (int i = 0; i < 7; ++i) f[i] = rec[i];
      const float gq = gout[qc];
      const int u = glint_wrap(f[0], a.nu);
      const int v = glint_wrap(f[1], a.nv);
      const int l = glint_clampi(f[2], 0, nl - 1);
      const int slo = glint_clampi(f[3], 0, a.N), shi = glint_clampi(f[4], 0, a.N);
      const int tlo = glint_clampi(f[5], 0, a.N), thi = glint_clampi(f[6], 0, a.N);
      const bool live = qi < a.nq && slo < shi && tlo < thi;
      QueryRows r;
      r.u = u * R;
      r.v = v * R;
      r.l = l * R;
      r.sh = shi * R;
      r.sl = slo * R;
      r.th = thi * R;
      r.tl = tlo * R;
      r.pad = __float_as_int(live ? gq : 0.0f);
      wrows[lane] = r;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    for (int jj = 0; jj < LPQ; ++jj) {
      const QueryRows r = wrows[g * LPQ + jj];
      const float gq = __int_as_float(r.pad);
      if (gq == 0.0f) continue;
      if (r.u != cu || r.v != cv || r.l != cl) {
        flush();
        cu = r.u; cv = r.v; cl = r.l;
      }
      float uu[RPL], vv[RPL], lr[RPL], sh[RPL], sl[RPL], th[RPL], tl[RPL];
      load_row<FT, RPL>(U + r.u + r0, uu);
      load_row<FT, RPL>(V + r.v + r0, vv);
      lds_row<RPL>(Ls + r.l + r0, lr);
      lds_row<RPL>(CSs + r.sh + r0, sh);
      lds_row<RPL>(CSs + r.sl + r0, sl);
      lds_row<RPL>(CTs + r.th + r0, th);
      lds_row<RPL>(CTs + r.tl + r0, tl);
#pragma unroll
      for (int e = 0; e < RPL; ++e) {
        const float s = scr[e] * gq;
        const float dS = sh[e] - sl[e];
        const float dT = th[e] - tl[e];
        const float st = dS * dT;
        const float uv = uu[e] * vv[e];
        aU[e] += s * vv[e] * lr[e] * st;
        aV[e] += s * uu[e] * lr[e] * st;
        aL[e] += s * uv * st;
        const float wS = s * uv * lr[e] * dT;
        const int sw = e * LPQ + j;
        atomicAdd(&gCS[r.sh + sw], wS);
        atomicAdd(&gCS[r.sl + sw], -wS);
        const float wT = s * uv * lr[e] * dS;
        atomicAdd(&gCT[r.th + sw], wT);
        atomicAdd(&gCT[r.tl + sw], -wT);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  flush();
  __syncthreads();
  // swizzled position p of a row holds rank (p % LPQ) * RPL + p / LPQ
  for (int i = threadIdx.x; i < nl * R; i += blockDim.x) {
    const int row = i / R, p = i % R;
    if (gL[i] != 0.0f) atomicAdd(&dL[row * R + (p % LPQ) * RPL + p / LPQ], gL[i]);
  }
  for (int i = threadIdx.x; i < N1 * R; i += blockDim.x) {
    const int row = i / R, p = i % R;
    const int k = row * R + (p % LPQ) * RPL + p / LPQ;
    if (gCS[i] != 0.0f) atomicAdd(&dCS[k], gCS[i]);
    if (gCT[i] != 0.0f) atomicAdd(&dCT[k], gCT[i]);
  }
}

// Query backward in the rank-owner layout, for N <= 64 (NT = ceil((N+1)/16)
// row tiles): wavefront w of a block owns ranks [16 w, 16 w + 16) and every
// wavefront walks the block's chunk of records four at a time, lane
// j + 16 k holding rank 16 w + j of record k.  The summed-area-table
// gradients dCS[row][r] = sum over records of ([row = s_hi] - [row = s_lo]) wS
// (and dCT, and dL over the levels) are products of a one-hot record-to-row
// matrix with the per-record rank vectors, so they accumulate on the matrix
// cores (v_mfma_f32_16x16x4f32: A[i][k] from lane i + 16k, B[k][j] from lane
// j + 16k) in registers for the whole chunk and reach global memory once per
// block.  dU and dV are summed over the records of a step that share the
// footprint and kept in registers while the footprint repeats.
typedef float bwd_f32x4 __attribute__((ext_vector_type(4)));

struct alignas(16) BwdRec {
  int u, v, l, sh, sl, th, tl;
  float g;
};

template <int NT>
constexpr bool backward_mfma_tiles_ok() { return NT >= 1 && NT <= 5; }

// waves of one record stream (one per 16-rank tile) and record streams per block
template <int R>
constexpr int bwd_streams() { return R / 16 >= 16 ? 1 : 16 / (R / 16); }

template <typename FT, typename CT, int R, int NT>
__global__ __launch_bounds__(1024) void k_query_backward_mfma(QueryArgs a, const float* __restrict__ gout,
                                                                     float* __restrict__ dU,
                                                                     float* __restrict__ dV,
                                                                     float* __restrict__ dL,
                                                                     float* __restrict__ dCS,
                                                                     float* __restrict__ dCT, int64_t chunk) {
  static_assert(backward_mfma_tiles_ok<NT>(), "row tiles");
  extern __shared__ __align__(16) float lds[];
  const int nl = a.nl, N1 = a.N + 1;
  float* Ls = lds;                  // decoded L (no scale)
  float* CSs = Ls + nl * R;
  float* CTs = CSs + N1 * R;
  float* sc = CTs + N1 * R;         // [R] folded scale
  BwdRec* slots = reinterpret_cast<BwdRec*>(sc + R);
  stage_table<FT>(Ls, static_cast<const FT*>(a.L), nl, R, nullptr);
  stage_table<CT>(CSs, static_cast<const CT*>(a.CS), N1, R, nullptr);
  stage_table<CT>(CTs, static_cast<const CT*>(a.CT), N1, R, nullptr);
  for (int i = threadIdx.x; i < R; i += blockDim.x) sc[i] = folded_scale(a.scale, i);
  __syncthreads();

  const FT* __restrict__ U = static_cast<const FT*>(a.U);
  const FT* __restrict__ V = static_cast<const FT*>(a.V);
  constexpr int NW = R / 16;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int w = wid % NW, stream = wid / NW;           // rank tile and record stream of this wave
  const int j = lane & 15, kq = lane >> 4;
  const int r = 16 * w + j;
  const float scr = sc[r];
  BwdRec* wslots = slots + wid * 64;
  bwd_f32x4 accS[NT], accT[NT], accL;
#pragma unroll
  for (int t = 0; t < NT; ++t) accS[t] = accT[t] = bwd_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  accL = bwd_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  int cu = -1, cv = -1;          // footprint of the running dU, dV sums (lanes of record slot 0)
  float ru = 0.0f, rv = 0.0f;
  auto flush = [&]() {
    if (kq == 0 && cu >= 0) {
      if (ru != 0.0f) atomicAdd(&dU[cu * R + r], ru);
      if (rv != 0.0f) atomicAdd(&dV[cv * R + r], rv);
    }
    cu = cv = -1;
    ru = rv = 0.0f;
  };
  const int64_t t0 = (static_cast<int64_t>(blockIdx.x) * bwd_streams<R>() + stream) * chunk;
  const int64_t t1 = t0 + chunk < a.nq ? t0 + chunk : a.nq;
  for (int64_t base = t0; base < t1; base += 64) {
    {
      const int64_t qi = base + lane;
      const bool in = qi < t1;
      const int64_t qc = in ? qi : t1 - 1;
      const int32_t* rec = a.q + qc * 7;
      int f[7];
#pragma unroll
      for (int i = 0; i < 7; ++i) f[i] = rec[i];
      const float gq = gout[qc];
      BwdRec b;
      b.u = glint_wrap(f[0], a.nu);
      b.v = glint_wrap(f[1], a.nv);
      b.l = glint_clampi(f[2], 0, nl - 1);
      const int slo = glint_clampi(f[3], 0, a.N), shi = glint_clampi(f[4], 0, a.N);
      const int tlo = glint_clampi(f[5], 0, a.N), thi = glint_clampi(f[6], 0, a.N);
      b.sh = shi; b.sl = slo; b.th = thi; b.tl = tlo;
      b.g = (in && slo < shi && tlo < thi) ? gq : 0.0f;
      wslots[lane] = b;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // the U and V values of the next step are loaded while this one is used
    BwdRec bn = wslots[kq];
    float un = dec<FT>(U[bn.u * R + r]), vn = dec<FT>(V[bn.v * R + r]);
    for (int st = 0; st < 16; ++st) {
      const BwdRec b = bn;
      const float uu = un, vv = vn;
      if (st < 15) {
        bn = wslots[4 * (st + 1) + kq];
        un = dec<FT>(U[bn.u * R + r]);
        vn = dec<FT>(V[bn.v * R + r]);
      }
      const float ll = Ls[b.l * R + r];
      const float dS = CSs[b.sh * R + r] - CSs[b.sl * R + r];
      const float dT = CTs[b.th * R + r] - CTs[b.tl * R + r];
      const float x = b.g * scr;
      const float uvl = uu * vv * ll;
      const float wS = x * uvl * dT, wT = x * uvl * dS;
      const float st2 = dS * dT;
      const float gu = x * vv * ll * st2, gv = x * uu * ll * st2, gl = x * uu * vv * st2;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int row = 16 * t + j;
        const float as = (row == b.sh ? 1.0f : 0.0f) - (row == b.sl ? 1.0f : 0.0f);
        const float at = (row == b.th ? 1.0f : 0.0f) - (row == b.tl ? 1.0f : 0.0f);
        accS[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(as, wS, accS[t], 0, 0, 0);
        accT[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(at, wT, accT[t], 0, 0, 0);
      }
      accL = __builtin_amdgcn_mfma_f32_16x16x4f32(j == b.l ? 1.0f : 0.0f, gl, accL, 0, 0, 0);
      // dU, dV: one sum per step when its four records share the footprint
      const int u0 = __shfl(b.u, j), v0 = __shfl(b.v, j);
      if (__all(b.u == u0 && b.v == v0)) {
        float su = gu + __shfl_xor(gu, 16), sv = gv + __shfl_xor(gv, 16);
        su += __shfl_xor(su, 32);
        sv += __shfl_xor(sv, 32);
        if (u0 != cu || v0 != cv) {
          flush();
          cu = u0;
          cv = v0;
        }
        ru += su;
        rv += sv;
      } else {
        flush();
        if (gu != 0.0f) atomicAdd(&dU[b.u * R + r], gu);
        if (gv != 0.0f) atomicAdd(&dV[b.v * R + r], gv);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  flush();
  // D[i][j] sits in lane j + 16 (i / 4), item i % 4
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = 16 * t + 4 * kq + q;
      if (row < N1) {
        if (accS[t][q] != 0.0f) atomicAdd(&dCS[row * R + r], accS[t][q]);
        if (accT[t][q] != 0.0f) atomicAdd(&dCT[row * R + r], accT[t][q]);
      }
    }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = 4 * kq + q;
    if (row < nl && accL[q] != 0.0f) atomicAdd(&dL[row * R + r], accL[q]);
  }
}

__global__ void k_fill(float* __restrict__ p, int64_t n, float v) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------
// summed-area tables and conversion
// ---------------------------------------------------------------------------

template <typename IN>
__device__ __forceinline__ double load_in(const IN* p, int64_t i) {
  return static_cast<double>(p[i]);
}

// Store an FP64 value into the output type (FP8 uses the column scale).
template <typename OUT>
__device__ __forceinline__ OUT enc(double x, float scale);
template <>
__device__ __forceinline__ double enc<double>(double x, float) { return x; }
template <>
__device__ __forceinline__ float enc<float>(double x, float) { return static_cast<float>(x); }
template <>
__device__ __forceinline__ uint16_t enc<uint16_t>(double x, float) {
  return glint_f32_to_bf16(static_cast<float>(x));
}
template <>
__device__ __forceinline__ uint8_t enc<uint8_t>(double x, float scale) {
  return static_cast<uint8_t>(glint_f32_to_fp8(static_cast<float>(x) / scale));
}

// One thread per column: C[j][r] = sum_{s<j} S[s][r] in FP64.
template <typename IN, typename OUT>
__global__ void k_cumulative(int n, int R, const IN* __restrict__ S, OUT* __restrict__ C,
                             float* __restrict__ col_scale) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  float scale = 1.0f;
  if constexpr (std::is_same<OUT, uint8_t>::value) {
    double acc = 0.0;
    float amax = 0.0f;
    for (int s = 0; s < n; ++s) {
      acc += load_in(S, static_cast<int64_t>(s) * R + r);
      amax = fmaxf(amax, fabsf(static_cast<float>(acc)));
    }
    scale = amax > 0.0f ? amax / 448.0f : 1.0f;
    col_scale[r] = scale;
  }
  double acc = 0.0;
  C[r] = enc<OUT>(0.0, scale);
  for (int s = 0; s < n; ++s) {
    acc += load_in(S, static_cast<int64_t>(s) * R + r);
    C[static_cast<int64_t>(s + 1) * R + r] = enc<OUT>(acc, scale);
  }
}

// Per-column amax of the FP32-rounded values, then the FP8 scale.
template <typename IN>
__global__ __launch_bounds__(256) void k_col_scale(int64_t rows, int R, const IN* __restrict__ in,
                                                   float* __restrict__ col_scale) {
  __shared__ float part[256];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int grp = threadIdx.x >> 6;
  float amax = 0.0f;
  if (c < R)
    for (int64_t i = grp; i < rows; i += 4)
      amax = fmaxf(amax, fabsf(static_cast<float>(in[i * R + c])));
  part[threadIdx.x] = amax;
  __syncthreads();
  if (grp == 0 && c < R) {
    amax = fmaxf(fmaxf(part[threadIdx.x], part[threadIdx.x + 64]),
                 fmaxf(part[threadIdx.x + 128], part[threadIdx.x + 192]));
    col_scale[c] = amax > 0.0f ? amax / 448.0f : 1.0f;
  }
}

template <typename IN, typename OUT>
__global__ void k_convert(int64_t n, int R, const IN* __restrict__ in, OUT* __restrict__ out,
                          const float* __restrict__ col_scale) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    float scale = 1.0f;
    if constexpr (std::is_same<OUT, uint8_t>::value) scale = col_scale[i % R];
    // every narrow type is reached through FP32 (FP64 -> FP32 -> narrow, each RNE)
    out[i] = enc<OUT>(static_cast<double>(static_cast<float>(in[i])), scale);
  }
}

__global__ void k_cumulative_backward(int n, int R, const float* __restrict__ dC,
                                      float* __restrict__ dS) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double acc = 0.0;
  for (int s = n - 1; s >= 0; --s) {
    acc += static_cast<double>(dC[static_cast<int64_t>(s + 1) * R + r]);
    dS[static_cast<int64_t>(s) * R + r] = static_cast<float>(acc);
  }
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------

int g_cu_count = 0;
int g_max_lds = 0;

glint_status device_limits() {
  if (g_cu_count > 0) return GLINT_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return glint_fail(GLINT_E_HIP, "hipGetDevice failed");
  int cus = 0, lds = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return glint_fail(GLINT_E_HIP, "hipDeviceGetAttribute failed");
  g_cu_count = cus;
  g_max_lds = lds;
  return GLINT_OK;
}

// Ranks per lane of a query group: each lane gathers 32 bytes of a factor row
// from rank 64 up (half the lanes per query, so the group reduction and the
// per-record bookkeeping are shared by twice as many queries per instruction;
// measured 1.0-1.5x faster there), 16 bytes below; never more than R.
// Rank 16 over FP32 tables small enough for LDS (U and V up to kRepRows
// rows): every 64-byte table row (L with the folded scales, CS, CT, U, V) is
// stored four times side by side, one copy in each quarter of the LDS banks,
// and the lane groups at positions 0..3 of a 16-lane LDS pass read copies
// 0..3, so the seven random rows of the four queries in a pass never share a
// bank (rows of one table otherwise start on one of four bank positions and
// collide about two ways) and the U and V gathers leave the texture
// address path.  Same arithmetic in the same order as k_query at rank 16.
constexpr int kRepRows = 128;

__host__ __device__ inline size_t rep16_lds_bytes(int nl, int N, int nu, int nv) {
  return sizeof(float) * 64 * (static_cast<size_t>(nl) + 2 * (static_cast<size_t>(N) + 1) + nu + nv) +
         sizeof(PackedRows) * 16 * (64 + 16);
}

__device__ void stage_rep16(float* __restrict__ dst, const float* __restrict__ src, int rows, const Scales* sc) {
  const int n = rows * 16;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    float x = src[i];
    if (sc) x *= folded_scale(*sc, i % 16);
    float* d = dst + (i / 16) * 64 + i % 16;
    d[0] = x;
    d[16] = x;
    d[32] = x;
    d[48] = x;
  }
}

__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_query_rep16(QueryArgs a) {
  constexpr int R = 16, RPL = 4, LPQ = 4, RW = 64, kSlots = 64 + 16;
  extern __shared__ __align__(16) float lds[];
  unsigned char* lds_b = reinterpret_cast<unsigned char*>(lds);
  float* Ls = lds;
  float* CSs = Ls + a.nl * RW;
  float* CTs = CSs + (a.N + 1) * RW;
  float* Us = CTs + (a.N + 1) * RW;
  float* Vs = Us + a.nu * RW;
  PackedRows* rows = reinterpret_cast<PackedRows*>(Vs + a.nv * RW);
  stage_rep16(Ls, static_cast<const float*>(a.L), a.nl, &a.scale);
  stage_rep16(CSs, static_cast<const float*>(a.CS), a.N + 1, nullptr);
  stage_rep16(CTs, static_cast<const float*>(a.CT), a.N + 1, nullptr);
  stage_rep16(Us, static_cast<const float*>(a.U), a.nu, nullptr);
  stage_rep16(Vs, static_cast<const float*>(a.V), a.nv, nullptr);
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int g = lane / LPQ;
  const int j = lane % LPQ;
  const int r0 = j * RPL + (g & 3) * R;   // the lane's columns in its group's copy
  PackedRows* wrows = rows + (threadIdx.x >> 6) * kSlots;
  const int my_slot = lane + lane / LPQ;
  const unsigned char* cum_lane = lds_b + r0 * sizeof(float);
  const uint32_t cs = static_cast<uint32_t>(reinterpret_cast<unsigned char*>(CSs) - lds_b);
  const uint32_t ct = static_cast<uint32_t>(reinterpret_cast<unsigned char*>(CTs) - lds_b);
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < a.nq; base += nwaves * 64) {
    {
      const int64_t qi = base + lane;
      const int64_t qc = qi < a.nq ? qi : a.nq - 1;
      const int32_t* rec = a.q + qc * 7;
      int f[7];
#pragma unroll
      for (int i = 0; i < 7; ++i) f[i] = __builtin_nontemporal_load(rec + i);
      const int u = glint_wrap(f[0], a.nu);
      const int v = glint_wrap(f[1], a.nv);
      const int l = glint_clampi(f[2], 0, a.nl - 1);
      const int slo = glint_clampi(f[3], 0, a.N), shi = glint_clampi(f[4], 0, a.N);
      const int tlo = glint_clampi(f[5], 0, a.N), thi = glint_clampi(f[6], 0, a.N);
      const bool empty = !(slo < shi && tlo < thi);
      const int s_hi = empty ? slo : shi;
      constexpr uint32_t RB = sizeof(float) * RW;
      PackedRows r;
      r.ul = static_cast<uint32_t>(u) | static_cast<uint32_t>(l) << 26;
      r.v = static_cast<uint32_t>(v);
      r.a = ((cs + s_hi * RB) >> 4) | ((cs + slo * RB) >> 4) << 16;
      r.b = ((ct + thi * RB) >> 4) | ((ct + tlo * RB) >> 4) << 16;
      wrows[my_slot] = r;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    float res = 0.0f;
    uint32_t pul = ~0u, pv = ~0u;
    float W[RPL];
#pragma unroll 2
    for (int jj = 0; jj < LPQ; ++jj) {
      const PackedRows r = wrows[g * (LPQ + 1) + jj];
      if (r.ul != pul || r.v != pv) {
        float uu[RPL], vv[RPL], lr[RPL];
        lds_row<RPL>(Us + (r.ul & 0x3ffffffu) * RW + r0, uu);
        lds_row<RPL>(Vs + r.v * RW + r0, vv);
        lds_row<RPL>(Ls + (r.ul >> 26) * RW + r0, lr);
#pragma unroll
        for (int e = 0; e < RPL; ++e) W[e] = uu[e] * vv[e] * lr[e];
        pul = r.ul; pv = r.v;
      }
      float sh[RPL], sl[RPL], th[RPL], tl[RPL];
      lds_row<RPL>(reinterpret_cast<const float*>(cum_lane + ((r.a & 0xffffu) << 4)), sh);
      lds_row<RPL>(reinterpret_cast<const float*>(cum_lane + ((r.a >> 16) << 4)), sl);
      lds_row<RPL>(reinterpret_cast<const float*>(cum_lane + ((r.b & 0xffffu) << 4)), th);
      lds_row<RPL>(reinterpret_cast<const float*>(cum_lane + ((r.b >> 16) << 4)), tl);
      float acc = lane_terms<RPL, RPL>(W, sh, sl, th, tl, 0);
      acc = glint_group_sum<LPQ>(acc);
      res = (j == jj) ? acc : res;
    }
    __builtin_amdgcn_wave_barrier();
    const int64_t qo = base + g * LPQ + j;
    if (qo < a.nq) __builtin_nontemporal_store(res, a.out + qo);
  }
}

template <typename FT, int R>
constexpr int rpl_for() {
  return (R >= 64 ? 32 : 16) / static_cast<int>(sizeof(FT)) <= R ? (R >= 64 ? 32 : 16) / static_cast<int>(sizeof(FT))
                                                                   : R;
}

template <typename CT>
size_t cum_lds_bytes(int N1, int R) {
  return 2 * sizeof(typename LdsCum<CT>::type) * static_cast<size_t>(N1) * R;
}

// LDS bytes of a query launch: L (FP32), the summed-area tables unless they
// are read from global memory, and the per-wave record slots.
template <typename CT, int R>
size_t query_lds_bytes(int nl, int N, bool global_cum, size_t slot_bytes) {
  return glint_round_up(sizeof(float) * static_cast<size_t>(nl) * R + (global_cum ? 0 : cum_lds_bytes<CT>(N + 1, R)),
                        16) + slot_bytes;
}

// The flat query's plan for a table type: ranks per lane and the element
// type of the LDS copies of the summed-area tables.  BF16 tables at rank 64
// take the FP32 layout (8 lanes per query, FP32 LDS copies): the BF16 factor
// rows halve the gathered bytes and the summed-area rows need no decoding in
// the loop (measured 10% faster than FP32 tables on pixel-coherent batches).
// Larger ranks keep BF16 LDS copies, whose FP32 copies would cost occupancy.
// FP32 tables from rank 128 up take 16 ranks (64 bytes) a lane: a wave then
// serves eight queries per step, halving the per-query share of the record
// read, the row-address arithmetic and the lane reduction, which bind there
// once the LDS reads are conflict-free (rank 128: 26.3 -> 33.0 G queries/s
// on the 2^24-record batch; rank 256 +11%; at ranks 16 and 64 the wider
// slices lost 30% and 20%).
template <typename FT, typename CT, int R>
struct QueryPlan {
  // BF16 factor tables at ranks 64 and 128 read their summed-area rows from
  // FP32 copies in LDS (decoded once per block: every BF16 or FP8 value is
  // exact in FP32), in the FP32 rank layout; measured on 2^24 rank-128
  // records with BF16 summed-area tables, 32.1 -> 38.0 G queries/s
  static constexpr bool kF32Lds = sizeof(FT) == 2 && (R == 64 || R == 128);
  static constexpr int RPL = kF32Lds ? (R == 128 ? 16 : 8) : ((sizeof(FT) == 4 && R >= 128) ? 16 : rpl_for<FT, R>());
  typedef typename std::conditional<kF32Lds, float, typename LdsCum<CT>::type>::type LT;
  // 1024-thread blocks where the kernel fits 64 VGPRs at little cost: FP32
  // factor rows up to rank 64 and the BF16 rank-64 layout (5% and 4% faster
  // at rank 64).  The rest keep 512: BF16 LDS rows at rank 128 spill and run
  // 7x slower, FP32 rank 128 is 2% slower, FP8 factor rows (32 ranks a lane)
  // would spill hundreds of bytes.
  static constexpr int NT =
      std::is_same<LT, float>::value && (sizeof(FT) == 4 ? R <= 64 : (sizeof(FT) == 2 && R == 64)) ? 1024
                                                                                                   : kQueryThreads;
};

template <typename FT, typename CT, int R>
glint_status launch_query(const QueryArgs& a, hipStream_t stream) {
  typedef QueryPlan<FT, CT, R> P;
  typedef typename P::LT LT;
  constexpr int RPL = P::RPL;
  // the packed records hold u in 26 bits and l in 6, LDS offsets / 16 in 16
  if (a.nu > (1 << 26) || a.nl > 64)
    return glint_fail(GLINT_E_UNSUPPORTED, "the flat query takes nu <= 2^26 and nl <= 64 (nu %d, nl %d)", a.nu, a.nl);
  constexpr int NT = P::NT;
  if constexpr (R == 16 && std::is_same<FT, float>::value && std::is_same<CT, float>::value) {
    const size_t rep = rep16_lds_bytes(a.nl, a.N, a.nu, a.nv);
    if (a.nu <= kRepRows && a.nv <= kRepRows && rep <= static_cast<size_t>(g_max_lds) &&
        16 * (static_cast<size_t>(a.nl) + 2 * (static_cast<size_t>(a.N) + 1)) < 65536) {
      const int64_t waves_needed = (a.nq + 63) / 64;
      int64_t blocks = (waves_needed + 15) / 16;
      const int64_t cap = static_cast<int64_t>(g_cu_count) * 2;
      if (blocks > cap) blocks = cap;
      if (blocks < 1) blocks = 1;
      glint_clear_launch_error();
      hipLaunchKernelGGL(k_query_rep16, dim3(static_cast<unsigned>(blocks)), dim3(1024), rep, stream, a);
      GLINT_LAUNCHED("k_query_rep16");
      return GLINT_OK;
    }
  }
  const size_t slots = sizeof(PackedRows) * (NT / 64) * (64 + 64 / (R / RPL));
  const bool gc = query_lds(a.nl, a.N, R, sizeof(LT), false, slots).total > static_cast<size_t>(g_max_lds);
  const size_t lds = query_lds(a.nl, a.N, R, sizeof(LT), gc, slots).total;
  if (lds > static_cast<size_t>(g_max_lds))
    return glint_fail(GLINT_E_UNSUPPORTED, "L needs %zu bytes of LDS (device max %d)", lds, g_max_lds);
  const int64_t waves_needed = (a.nq + 63) / 64;
  constexpr int WPB = NT / 64;
  int64_t blocks = (waves_needed + WPB - 1) / WPB;
  const int64_t cap = static_cast<int64_t>(g_cu_count) * (2048 / NT);
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  glint_clear_launch_error();
  const dim3 grid(static_cast<unsigned>(blocks)), block(NT);
  if (gc)
    hipLaunchKernelGGL((k_query<FT, CT, LT, R, RPL, true, NT>), grid, block, lds, stream, a);
  else
    hipLaunchKernelGGL((k_query<FT, CT, LT, R, RPL, false, NT>), grid, block, lds, stream, a);
  GLINT_LAUNCHED("k_query");
  return GLINT_OK;
}

template <typename FT, typename CT, int R>
glint_status launch_grouped(const GroupedArgs& a, hipStream_t stream) {
  // FP8 factor rows at rank 256 (the summed-area copies in LDS take 132 KB, one
  // block a CU): 16 ranks a lane in a 1024-thread block, four waves a SIMD
  // instead of two at 128 VGPRs (52 bytes of spill); with the box records
  // loaded one box ahead, 2^20 points x 32 boxes 13.7 -> 15.7 G boxes/s
  constexpr bool kWide = sizeof(FT) == 1 && R == 256;
  constexpr int RPL = kWide ? 16 : rpl_for<FT, R>();
  constexpr int NT = kWide ? 1024 : kQueryThreads;
  const size_t slots = sizeof(int4) * (NT / 64) * 64;
  const bool gc = static_cast<int>(query_lds_bytes<CT, R>(a.nl, a.N, false, slots)) > g_max_lds;
  const size_t lds = query_lds_bytes<CT, R>(a.nl, a.N, gc, slots);
  if (static_cast<int>(lds) > g_max_lds)
    return glint_fail(GLINT_E_UNSUPPORTED, "L needs %zu bytes of LDS (device max %d)", lds, g_max_lds);
  const int64_t waves_needed = (a.npts + 63) / 64;
  constexpr int WPB = NT / 64;
  int64_t blocks = (waves_needed + WPB - 1) / WPB;
  const int64_t cap = static_cast<int64_t>(g_cu_count) * (2048 / NT);
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  glint_clear_launch_error();
  if (gc)
    hipLaunchKernelGGL((k_query_grouped<FT, CT, R, RPL, true, NT>), dim3(static_cast<unsigned>(blocks)),
                       dim3(NT), lds, stream, a);
  else
    hipLaunchKernelGGL((k_query_grouped<FT, CT, R, RPL, false, NT>), dim3(static_cast<unsigned>(blocks)),
                       dim3(NT), lds, stream, a);
  GLINT_LAUNCHED("k_query_grouped");
  return GLINT_OK;
}

template <typename FT, typename CT, int R>
glint_status launch_trilinear(const TriArgs& a, hipStream_t stream) {
  constexpr int RPL = rpl_for<FT, R>();
  // the packed records hold u in 26 bits and l in 6
  if (a.nu > (1 << 26) || a.nl > 64)
    return glint_fail(GLINT_E_UNSUPPORTED, "the trilinear query takes nu <= 2^26 and nl <= 64 (nu %d, nl %d)", a.nu,
                      a.nl);
  const size_t slots = sizeof(TriRows) * (kQueryThreads / 64) * (64 + 64 / (R / RPL));
  const bool gc = static_cast<int>(query_lds_bytes<CT, R>(a.nl, a.N, false, slots)) > g_max_lds;
  const size_t lds = query_lds_bytes<CT, R>(a.nl, a.N, gc, slots);
  if (static_cast<int>(lds) > g_max_lds)
    return glint_fail(GLINT_E_UNSUPPORTED, "L needs %zu bytes of LDS (device max %d)", lds, g_max_lds);
  const int64_t waves_needed = (a.nq + 63) / 64;
  constexpr int WPB = kQueryThreads / 64;
  int64_t blocks = (waves_needed + WPB - 1) / WPB;
  const int64_t cap = static_cast<int64_t>(g_cu_count) * 4;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  glint_clear_launch_error();
  if (gc)
    hipLaunchKernelGGL((k_query_trilinear<FT, CT, R, RPL, true>), dim3(static_cast<unsigned>(blocks)),
                       dim3(kQueryThreads), lds, stream, a);
  else
    hipLaunchKernelGGL((k_query_trilinear<FT, CT, R, RPL, false>), dim3(static_cast<unsigned>(blocks)),
                       dim3(kQueryThreads), lds, stream, a);
  GLINT_LAUNCHED("k_query_trilinear");
  return GLINT_OK;
}

template <typename FT, typename CT, int R>
glint_status launch_sample(const SampleArgs& a, hipStream_t stream) {
  constexpr int RPL = rpl_for<FT, R>();
  const size_t slots = sizeof(int4) * (kQueryThreads / 64) * 64;
  const bool gc = static_cast<int>(query_lds_bytes<CT, R>(a.nl, a.N, false, slots)) > g_max_lds;
  const size_t lds = query_lds_bytes<CT, R>(a.nl, a.N, gc, slots);
  if (static_cast<int>(lds) > g_max_lds)
    return glint_fail(GLINT_E_UNSUPPORTED, "L needs %zu bytes of LDS (device max %d)", lds, g_max_lds);
  const int64_t waves_needed = (a.n + 63) / 64;
  constexpr int WPB = kQueryThreads / 64;
  int64_t blocks = (waves_needed + WPB - 1) / WPB;
  const int64_t cap = static_cast<int64_t>(g_cu_count) * 4;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  glint_clear_launch_error();
  if (gc)
    hipLaunchKernelGGL((k_sample<FT, CT, R, RPL, true>), dim3(static_cast<unsigned>(blocks)), dim3(kQueryThreads),
                       lds, stream, a);
  else
    hipLaunchKernelGGL((k_sample<FT, CT, R, RPL, false>), dim3(static_cast<unsigned>(blocks)), dim3(kQueryThreads),
                       lds, stream, a);
  GLINT_LAUNCHED("k_sample");
  return GLINT_OK;
}

template <typename FT, typename CT, int R, int NT>
glint_status launch_backward_mfma(const QueryArgs& a, const float* gout, float* dU, float* dV, float* dL,
                                  float* dCS, float* dCT, hipStream_t stream) {
  constexpr int NW = R / 16, NS = bwd_streams<R>();
  const size_t lds = sizeof(float) * (static_cast<size_t>(a.nl + 2 * (a.N + 1)) * R + R) +
                     sizeof(BwdRec) * NW * NS * 64;
  if (static_cast<int>(lds) > g_max_lds)
    return glint_fail(GLINT_E_UNSUPPORTED, "backward needs %zu bytes of LDS (device max %d)", lds, g_max_lds);
  // record streams of 64-record units, each a contiguous chunk
  const int64_t units = (a.nq + 63) / 64;
  int64_t streams = static_cast<int64_t>(g_cu_count) * 2 * NS;
  if (streams > units) streams = units;
  if (streams < 1) streams = 1;
  const int64_t chunk = (units + streams - 1) / streams * 64;
  streams = (a.nq + chunk - 1) / chunk;
  const int64_t blocks = (streams + NS - 1) / NS;
  glint_clear_launch_error();
  hipLaunchKernelGGL((k_query_backward_mfma<FT, CT, R, NT>), dim3(static_cast<unsigned>(blocks)), dim3(NW * NS * 64),
                     lds, stream, a, gout, dU, dV, dL, dCS, dCT, chunk);
  GLINT_LAUNCHED("k_query_backward_mfma");
  return GLINT_OK;
}

template <typename FT, typename CT, int R>
glint_status launch_backward(const QueryArgs& a, const float* gout, float* dU, float* dV,
                             float* dL, float* dCS, float* dCT, hipStream_t stream) {
  if (a.nl <= 16 && a.N <= 64) {
    switch ((a.N + 1 + 15) / 16) {
      case 1: return launch_backward_mfma<FT, CT, R, 1>(a, gout, dU, dV, dL, dCS, dCT, stream);
      case 2: return launch_backward_mfma<FT, CT, R, 2>(a, gout, dU, dV, dL, dCS, dCT, stream);
      case 3: return launch_backward_mfma<FT, CT, R, 3>(a, gout, dU, dV, dL, dCS, dCT, stream);
      default: return launch_backward_mfma<FT, CT, R, 5>(a, gout, dU, dV, dL, dCS, dCT, stream);
    }
  }
  constexpr int RPL = rpl_for<FT, R>();
  const size_t lds = sizeof(float) * (2 * static_cast<size_t>(a.nl + 2 * (a.N + 1)) * R + R) +
                     sizeof(QueryRows) * (kQueryThreads / 64) * 64;
  if (static_cast<int>(lds) > g_max_lds)
    return glint_fail(GLINT_E_UNSUPPORTED, "backward needs %zu bytes of LDS (device max %d)", lds, g_max_lds);
  const int64_t waves_needed = (a.nq + 63) / 64;
  constexpr int WPB = kQueryThreads / 64;
  int64_t blocks = (waves_needed + WPB - 1) / WPB;
  const int64_t cap = static_cast<int64_t>(g_cu_count) * 2;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  glint_clear_launch_error();
  hipLaunchKernelGGL((k_query_backward<FT, CT, R, RPL>), dim3(static_cast<unsigned>(blocks)),
                     dim3(kQueryThreads), lds, stream, a, gout, dU, dV, dL, dCS, dCT);
  GLINT_LAUNCHED("k_query_backward");
  return GLINT_OK;
}

// R -> template argument
template <typename FT, typename CT, typename Fn>
glint_status by_rank(int R, Fn&& fn) {
  switch (R) {
    case 16: return fn(std::integral_constant<int, 16>{});
    case 32: return fn(std::integral_constant<int, 32>{});
    case 64: return fn(std::integral_constant<int, 64>{});
    case 128: return fn(std::integral_constant<int, 128>{});
    case 256: return fn(std::integral_constant<int, 256>{});
  }
  return glint_fail(GLINT_E_UNSUPPORTED, "rank %d not in {16,32,64,128,256}", R);
}

template <typename Fn>
glint_status by_types(glint_dtype ft, glint_dtype ct, Fn&& fn) {
  auto with_ct = [&](auto ftag) -> glint_status {
    using FT = decltype(ftag);
    switch (ct) {
      case GLINT_F32: return fn(FT{}, float{});
      case GLINT_BF16: return fn(FT{}, uint16_t{});
      case GLINT_FP8E4M3: return fn(FT{}, uint8_t{});
      default: break;
    }
    return glint_fail(GLINT_E_UNSUPPORTED, "cumulative-table dtype %d", static_cast<int>(ct));
  };
  switch (ft) {
    case GLINT_F32: return with_ct(float{});
    case GLINT_BF16: return with_ct(uint16_t{});
    case GLINT_FP8E4M3: return with_ct(uint8_t{});
    default: break;
  }
  return glint_fail(GLINT_E_UNSUPPORTED, "factor dtype %d", static_cast<int>(ft));
}

glint_status check_factors(const glint_factors* f) {
  GLINT_REQUIRE(f != nullptr, "factors is NULL");
  GLINT_REQUIRE(f->U && f->V && f->L && f->CS && f->CT, "null factor table");
  GLINT_REQUIRE(f->nu >= 1 && f->nv >= 1 && f->nl >= 1, "table sizes must be positive");
  GLINT_REQUIRE(glint_pow2(f->nbins) && f->nbins >= 4 && f->nbins <= 256,
                "nbins %d must be a power of two in 4..256", f->nbins);
  GLINT_REQUIRE(glint_aligned(f->U, 16) && glint_aligned(f->V, 16) && glint_aligned(f->L, 16) &&
                    glint_aligned(f->CS, 16) && glint_aligned(f->CT, 16),
                "factor tables must be 16-byte aligned");
  return device_limits();
}

Scales scales_of(const glint_factors* f) {
  Scales s;
  s.s[0] = f->scale_U; s.s[1] = f->scale_V; s.s[2] = f->scale_L;
  s.s[3] = f->scale_CS; s.s[4] = f->scale_CT;
  return s;
}

QueryArgs make_args(const glint_factors* f, int64_t nq, const int32_t* q, float* out) {
  QueryArgs a;
  a.U = f->U; a.V = f->V; a.L = f->L; a.CS = f->CS; a.CT = f->CT; a.scale = scales_of(f);
  a.nu = f->nu; a.nv = f->nv; a.nl = f->nl; a.N = f->nbins;
  a.nq = nq; a.q = q; a.out = out;
  return a;
}

}  // namespace

extern "C" {

glint_status glint_query(const glint_factors* f, int64_t nq, const int32_t* q, float* out,
                         hipStream_t stream) {
  glint_status st = check_factors(f);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(nq >= 0, "nq must be >= 0");
  if (nq == 0) return GLINT_OK;
  GLINT_REQUIRE(q && out, "null query or output pointer");
  const QueryArgs a = make_args(f, nq, q, out);
  return by_types(f->dtype, f->cum_dtype, [&](auto ft, auto ct) -> glint_status {
    using FT = decltype(ft);
    using CT = decltype(ct);
    return by_rank<FT, CT>(f->R, [&](auto rr) -> glint_status {
      return launch_query<FT, CT, decltype(rr)::value>(a, stream);
    });
  });
}

glint_status glint_query_trilinear(const glint_factors* f, int64_t nq, const float* xyl, const int32_t* boxes,
                                   float* out, hipStream_t stream) {
  glint_status st = check_factors(f);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(nq >= 0, "nq must be >= 0");
  if (nq == 0) return GLINT_OK;
  GLINT_REQUIRE(xyl && boxes && out, "null pointer argument");
  TriArgs a;
  a.U = f->U; a.V = f->V; a.L = f->L; a.CS = f->CS; a.CT = f->CT; a.scale = scales_of(f);
  a.nu = f->nu; a.nv = f->nv; a.nl = f->nl; a.N = f->nbins;
  a.nq = nq; a.xyl = xyl; a.boxes = boxes; a.out = out;
  return by_types(f->dtype, f->cum_dtype, [&](auto ft, auto ct) -> glint_status {
    using FT = decltype(ft);
    using CT = decltype(ct);
    return by_rank<FT, CT>(f->R, [&](auto rr) -> glint_status {
      return launch_trilinear<FT, CT, decltype(rr)::value>(a, stream);
    });
  });
}

glint_status glint_sample(const glint_factors* f, int64_t n, const int32_t* uvl, const float* rnd, float* h,
                          float* pdf, int32_t* bins, hipStream_t stream) {
  glint_status st = check_factors(f);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(n >= 0, "n must be >= 0");
  if (n == 0) return GLINT_OK;
  GLINT_REQUIRE(uvl && rnd && h && pdf && bins, "null pointer argument");
  SampleArgs a;
  a.U = f->U; a.V = f->V; a.L = f->L; a.CS = f->CS; a.CT = f->CT; a.scale = scales_of(f);
  a.nu = f->nu; a.nv = f->nv; a.nl = f->nl; a.N = f->nbins;
  a.levels = 0;
  while ((2 << a.levels) <= f->nbins) ++a.levels;     // log2(nbins)
  a.n = n; a.uvl = uvl; a.rnd = rnd; a.h = h; a.pdf = pdf; a.bins = bins;
  return by_types(f->dtype, f->cum_dtype, [&](auto ft, auto ct) -> glint_status {
    using FT = decltype(ft);
    using CT = decltype(ct);
    return by_rank<FT, CT>(f->R, [&](auto rr) -> glint_status {
      return launch_sample<FT, CT, decltype(rr)::value>(a, stream);
    });
  });
}

glint_status glint_query_grouped(const glint_factors* f, int64_t npts, int32_t K,
                                 const int32_t* uvl, const int32_t* boxes, float* out,
                                 hipStream_t stream) {
  glint_status st = check_factors(f);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(npts >= 0 && K >= 1, "npts must be >= 0 and K >= 1");
  if (npts == 0) return GLINT_OK;
  GLINT_REQUIRE(uvl && boxes && out, "null pointer argument");
  GLINT_REQUIRE(glint_aligned(boxes, 16), "boxes must be 16-byte aligned");
  GroupedArgs a;
  a.U = f->U; a.V = f->V; a.L = f->L; a.CS = f->CS; a.CT = f->CT; a.scale = scales_of(f);
  a.nu = f->nu; a.nv = f->nv; a.nl = f->nl; a.N = f->nbins; a.K = K;
  a.npts = npts; a.uvl = uvl; a.boxes = boxes; a.out = out;
  return by_types(f->dtype, f->cum_dtype, [&](auto ft, auto ct) -> glint_status {
    using FT = decltype(ft);
    using CT = decltype(ct);
    return by_rank<FT, CT>(f->R, [&](auto rr) -> glint_status {
      return launch_grouped<FT, CT, decltype(rr)::value>(a, stream);
    });
  });
}

glint_status glint_query_backward(const glint_factors* f, int64_t nq, const int32_t* q,
                                  const float* gout, float* dU, float* dV, float* dL,
                                  float* dCS, float* dCT, hipStream_t stream) {
  glint_status st = check_factors(f);
  if (st != GLINT_OK) return st;
  GLINT_REQUIRE(nq >= 0, "nq must be >= 0");
  GLINT_REQUIRE(dU && dV && dL && dCS && dCT, "null gradient pointer");
  GLINT_SUPPORT((f->dtype == GLINT_F32 || f->dtype == GLINT_BF16) &&
                    (f->cum_dtype == GLINT_F32 || f->cum_dtype == GLINT_BF16),
                "backward supports F32 and BF16 tables");
  const int R = f->R;
  struct { float* p; int64_t n; } bufs[5] = {
      {dU, static_cast<int64_t>(f->nu) * R}, {dV, static_cast<int64_t>(f->nv) * R},
      {dL, static_cast<int64_t>(f->nl) * R}, {dCS, static_cast<int64_t>(f->nbins + 1) * R},
      {dCT, static_cast<int64_t>(f->nbins + 1) * R}};
  for (auto& b : bufs) {
    glint_clear_launch_error();
    const int64_t blocks = (b.n + 255) / 256 < 1024 ? (b.n + 255) / 256 : 1024;
    hipLaunchKernelGGL(k_fill, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, b.p, b.n, 0.0f);
    GLINT_LAUNCHED("k_fill");
  }
  if (nq == 0) return GLINT_OK;
  GLINT_REQUIRE(q && gout, "null query or gout pointer");
  const QueryArgs a = make_args(f, nq, q, nullptr);
  return by_types(f->dtype, f->cum_dtype, [&](auto ft, auto ct) -> glint_status {
    using FT = decltype(ft);
    using CT = decltype(ct);
    if constexpr (std::is_same<FT, uint8_t>::value || std::is_same<CT, uint8_t>::value) {
      return glint_fail(GLINT_E_UNSUPPORTED, "backward supports F32 and BF16 tables");
    } else {
      return by_rank<FT, CT>(f->R, [&](auto rr) -> glint_status {
        return launch_backward<FT, CT, decltype(rr)::value>(a, gout, dU, dV, dL, dCS, dCT, stream);
      });
    }
  });
}

glint_status glint_cumulative_backward(int32_t n, int32_t R, const float* dC, float* dS,
                                       hipStream_t stream) {
  GLINT_REQUIRE(n >= 1 && R >= 1, "sizes must be positive");
  GLINT_REQUIRE(dC && dS, "null pointer argument");
  glint_clear_launch_error();
  hipLaunchKernelGGL(k_cumulative_backward, dim3((R + 255) / 256), dim3(256), 0, stream, n, R, dC, dS);
  GLINT_LAUNCHED("k_cumulative_backward");
  return GLINT_OK;
}

glint_status glint_make_cumulative(int32_t n, int32_t R, const void* S, glint_dtype in_dtype,
                                   void* C, glint_dtype out_dtype, float* col_scale,
                                   hipStream_t stream) {
  GLINT_REQUIRE(n >= 1 && R >= 1, "sizes must be positive");
  GLINT_REQUIRE(S && C, "null pointer argument");
  GLINT_REQUIRE(out_dtype != GLINT_FP8E4M3 || col_scale, "FP8 output needs col_scale");
  GLINT_SUPPORT(in_dtype == GLINT_F64 || in_dtype == GLINT_F32, "input dtype must be F64 or F32");
  const dim3 grid((R + 63) / 64), block(64);
  auto go = [&](auto in_tag) -> glint_status {
    using IN = decltype(in_tag);
    const IN* s = static_cast<const IN*>(S);
    glint_clear_launch_error();
    switch (out_dtype) {
      case GLINT_F64:
        hipLaunchKernelGGL((k_cumulative<IN, double>), grid, block, 0, stream, n, R, s,
                           static_cast<double*>(C), col_scale);
        break;
      case GLINT_F32:
        hipLaunchKernelGGL((k_cumulative<IN, float>), grid, block, 0, stream, n, R, s,
                           static_cast<float*>(C), col_scale);
        break;
      case GLINT_BF16:
        hipLaunchKernelGGL((k_cumulative<IN, uint16_t>), grid, block, 0, stream, n, R, s,
                           static_cast<uint16_t*>(C), col_scale);
        break;
      case GLINT_FP8E4M3:
        hipLaunchKernelGGL((k_cumulative<IN, uint8_t>), grid, block, 0, stream, n, R, s,
                           static_cast<uint8_t*>(C), col_scale);
        break;
      default:
        return glint_fail(GLINT_E_UNSUPPORTED, "output dtype %d", static_cast<int>(out_dtype));
    }
    GLINT_LAUNCHED("k_cumulative");
    return GLINT_OK;
  };
  if (in_dtype == GLINT_F64) return go(double{});
  return go(float{});
}

glint_status glint_convert(int64_t rows, int32_t R, const void* in, glint_dtype in_dtype,
                           void* out, glint_dtype out_dtype, float* col_scale,
                           hipStream_t stream) {
  GLINT_REQUIRE(rows >= 1 && R >= 1, "sizes must be positive");
  GLINT_REQUIRE(in && out, "null pointer argument");
  GLINT_REQUIRE(out_dtype != GLINT_FP8E4M3 || col_scale, "FP8 output needs col_scale");
  GLINT_SUPPORT(in_dtype == GLINT_F64 || in_dtype == GLINT_F32, "input dtype must be F64 or F32");
  GLINT_SUPPORT(out_dtype == GLINT_F32 || out_dtype == GLINT_BF16 || out_dtype == GLINT_FP8E4M3,
                "output dtype must be F32, BF16 or FP8E4M3");
  const int64_t n = rows * R;
  const unsigned blocks = static_cast<unsigned>((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  auto go = [&](auto in_tag) -> glint_status {
    using IN = decltype(in_tag);
    const IN* src = static_cast<const IN*>(in);
    glint_clear_launch_error();
    if (out_dtype == GLINT_FP8E4M3) {
      hipLaunchKernelGGL((k_col_scale<IN>), dim3((R + 63) / 64), dim3(256), 0, stream, rows, R, src, col_scale);
      GLINT_LAUNCHED("k_col_scale");
      hipLaunchKernelGGL((k_convert<IN, uint8_t>), dim3(blocks), dim3(256), 0, stream, n, R, src,
                         static_cast<uint8_t*>(out), col_scale);
    } else if (out_dtype == GLINT_BF16) {
      hipLaunchKernelGGL((k_convert<IN, uint16_t>), dim3(blocks), dim3(256), 0, stream, n, R, src,
                         static_cast<uint16_t*>(out), col_scale);
    } else {
      hipLaunchKernelGGL((k_convert<IN, float>), dim3(blocks), dim3(256), 0, stream, n, R, src,
                         static_cast<float*>(out), col_scale);
    }
    GLINT_LAUNCHED("k_convert");
    return GLINT_OK;
  };
  if (in_dtype == GLINT_F64) return go(double{});
  return go(float{});
}

}  // extern "C"
