// Pieces shared by the all-pairs screen kernels (FP32 and BF16x3 Grams):
// tile enumeration, the per-pair bounds of the epilogue, arg-reductions.
#pragma once
#include <type_traits>

#include "common.h"

namespace adg {

struct TilePos {
  int64_t I, J;
};

// Tile t of the row-major enumeration of the upper triangle I <= J < NT
// (row I starts at I*NT - I*(I-1)/2).
__device__ inline TilePos tri_tile_p(int64_t t, int64_t NT) {
  double b = 2.0 * (double)NT + 1.0;
  int64_t i = (int64_t)((b - sqrt(b * b - 8.0 * (double)t)) * 0.5);
  if (i < 0) i = 0;
  if (i > NT - 1) i = NT - 1;
  while (i > 0 && i * NT - i * (i - 1) / 2 > t) --i;
  while (i + 1 < NT && (i + 1) * NT - (i + 1) * i / 2 <= t) ++i;
  return TilePos{i, i + (t - (i * NT - i * (i - 1) / 2))};
}

// Slot -> tile (I, J) of the super-tiled upper triangle; I = -1 when the
// slot holds no tile.  NS = number of super-tile rows.
__device__ inline TilePos slot_tile(int64_t slot, int NT, int NS) {
  const TilePos S = tri_tile_p(slot >> 6, NS);
  const int loc = (int)(slot & 63);
  const int64_t I = S.I * 8 + (loc >> 3), J = S.J * 8 + (loc & 7);
  if (I <= J && J < NT) return TilePos{I, J};
  return TilePos{-1, -1};
}

__device__ inline bool idx_better(int ia, int ja, int ib, int jb) {
  return ia != ib ? ia < ib : ja < jb;
}

// (v, i, j): larger v wins (MAX) or smaller v wins (!MAX); ties -> smaller (i, j).
template <bool MAX>
__device__ inline void wave_arg(float& v, int& i, int& j) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const float v2 = __shfl_xor(v, o, 64);
    const int i2 = __shfl_xor(i, o, 64), j2 = __shfl_xor(j, o, 64);
    const bool take = MAX ? (v2 > v || (v2 == v && idx_better(i2, j2, i, j)))
                          : (v2 < v || (v2 == v && idx_better(i2, j2, i, j)));
    if (take) { v = v2; i = i2; j = j2; }
  }
}

// Point-Gram cache of a screen: the 16384 FP32 values of a 128 x 128 tile's
// point Gram (the accX accumulators of its 256 threads) stored as 16 float4
// per thread, element k4 of thread tid at float4 index k4 * 256 + tid of the
// tile's 64 KB block, so every store and load of a wave is one contiguous
// 1 KB segment.  The points do not change across the certificates of one
// fit, so the first certificate stores the Grams and the others load them.
// Every tile is written once and read once per screen: non-temporal stores
// and loads, so that the stream of cache blocks does not evict the row and
// column panels that neighbouring tiles share in L2.
__device__ inline void gcache_store(float* cache, int64_t tile, const f32x16 (&acc)[2][2]) {
  f32x4* g = reinterpret_cast<f32x4*>(cache) + tile * 4096 + threadIdx.x;
#pragma unroll
  for (int k4 = 0; k4 < 16; ++k4) {
    const f32x16& a = acc[k4 >> 3][(k4 >> 2) & 1];
    const int v = (k4 & 3) * 4;
    const f32x4 t = {a[v], a[v + 1], a[v + 2], a[v + 3]};
    __builtin_nontemporal_store(t, g + k4 * 256);
  }
}
__device__ inline void gcache_load(const float* cache, int64_t tile, f32x16 (&acc)[2][2]) {
  const f32x4* g = reinterpret_cast<const f32x4*>(cache) + tile * 4096 + threadIdx.x;
#pragma unroll
  for (int k4 = 0; k4 < 16; ++k4) {
    const f32x4 t = __builtin_nontemporal_load(g + k4 * 256);
    f32x16& a = acc[k4 >> 3][(k4 >> 2) & 1];
    const int v = (k4 & 3) * 4;
    a[v] = t[0]; a[v + 1] = t[1]; a[v + 2] = t[2]; a[v + 3] = t[3];
  }
}
// Compact cache block of a precision-form fit.  Per tile and pair, from the
// fill's D2lo (the FP32 lower bound on D^2 that the epilogue forms from the
// point Gram and its row terms), the FP16 value
//   g = c / D2lo rounded up
// (+infinity when D2lo <= c 2^-16 or the quotient passes 65504, so only for
// D2lo < c 2^-15), with c the fit's power of two, 2^-12 max N < c <=
// 2^-11 max N: every D2lo <= D^2 <= 4 max N then gives g > 2^-14, an FP16
// normal.  A finite g satisfies g >= c / D2lo (so
// q <= E2hi g / c) and D2lo <= (1 + 2^-10 + 2^-20) c / g (FP16 keeps 11
// significant bits; the 2^-20 covers the division's rounding and the
// inflation before the FP16 rounding).  32 KB per tile instead of 64, and the
// screens' fast pass needs no reciprocal.  Thread tid's 64 values sit in
// 16-byte slots k8 * 256 + tid (k8 = 0..7): slot k8 holds registers
// (k8 & 1) * 8 .. + 7 of accumulator block [k8 >> 2][(k8 >> 1) & 1], two per
// 32-bit word, the lower-numbered register in the low half.
__device__ inline uint32_t f16_up_bits(float x) {   // x > 0
  const _Float16 h = (_Float16)x;                    // nearest even (infinity past 65520)
  uint32_t b = __builtin_bit_cast(uint16_t, h);
  if ((float)h < x) ++b;                             // the next FP16 value up (0x7BFF + 1 = infinity)
  return b;
}
__device__ inline uint32_t dcache_code(float d2lo, float c) {
  if (!(d2lo > c * 0x1p-16f)) return 0x7C00u;        // +infinity: D2lo small, zero or negative
  return f16_up_bits((c / d2lo) * (1.0f + 0x1p-22f));
}
// The 8 slots of thread slot_tid of a tile's block, from that thread's 64
// D2lo values (in the order of its accumulators).
__device__ inline void dcache_store(void* cache, int64_t tile, const f32x16 (&d2lo)[2][2], float c, int slot_tid) {
  u32x4* g = reinterpret_cast<u32x4*>(cache) + tile * 2048 + slot_tid;
#pragma unroll
  for (int k8 = 0; k8 < 8; ++k8) {
    const f32x16& a = d2lo[k8 >> 2][(k8 >> 1) & 1];
    const int v = (k8 & 1) * 8;
    u32x4 t;
#pragma unroll
    for (int w = 0; w < 4; ++w) t[w] = dcache_code(a[v + 2 * w], c) | (dcache_code(a[v + 2 * w + 1], c) << 16);
    __builtin_nontemporal_store(t, g + k8 * 256);
  }
}
// The 8 slots of thread slot_tid of a tile's block into registers, still
// packed (32 registers).
__device__ inline void dcache_load(const void* cache, int64_t tile, u32x4 (&pk)[8], int slot_tid) {
  const u32x4* g = reinterpret_cast<const u32x4*>(cache) + tile * 2048 + slot_tid;
#pragma unroll
  for (int k8 = 0; k8 < 8; ++k8) pk[k8] = __builtin_nontemporal_load(g + k8 * 256);
}
// g of accumulator register v of block [x][y], as FP32 (exact).
__device__ inline float dcache_g(const u32x4 (&pk)[8], int x, int y, int v) {
  const uint32_t word = pk[x * 4 + y * 2 + (v >> 3)][(v & 7) >> 1];
  const uint16_t hb = (uint16_t)((v & 1) ? (word >> 16) : (word & 0xFFFFu));
  return (float)__builtin_bit_cast(_Float16, hb);
}

struct PairsArgs {
  const float* X; int ldx; int nchx;   // centred points, n_pad x ldx, ldx = 16 * nchx
  const float* Y; int ldy; int nchy;   // centred images, n_pad x ldy
  const float2* tx; const float2* ty;  // per-row (lo, hi) terms of D^2 and E^2
  int n; int NT; int64_t ntiles;
  int NS; int64_t nslots;              // super-tile rows, slots (64 per super-tile)
  TileRec* recs;                       // MODE 0, indexed by slot
  const uint32_t* list;                // MODE 1: flagged tiles
  const CertDev* cd;                   //         thresholds and count
  int2* cand; uint32_t cap; uint32_t* ncand;
  float* gcache; int gmode;            // MODE 0: point Gram per tile, 0 off, 1 store, 2 load
  // MODE 0 early stop (null: off): a pair with q_lo > stop_hi or q_hi <
  // stop_lo is certain to exceed the search's target; the pair goes to
  // stop_pairs[*stop] (first 8 kept), *stop counts them, and workgroups that
  // start after *stop became nonzero skip their tile.
  uint32_t* stop; int2* stop_pairs; float stop_hi, stop_lo;
  // compact D^2 cache (precision-form screens): device pointer to its scale
  // (null: gcache, if any, holds FP32 point Grams)
  const float* dscale;
};

// Bounds on q for one pair from its two Gram entries and row terms.  Branch
// free.  Identical points (D^2 upper bound <= 0, so D^2 = 0) get the neutral
// q = 1.  A D^2 bound at or below 1e-30 gives the widest bounds (q_hi = 3e38,
// q_lo = 0), so the pair is always re-examined.  Above it both reciprocals are
// finite and the products are never 0 * inf: no NaN can hide a pair.
__device__ inline void pair_bounds(float gx, float gy, const float4& ta, const float4& tb, float& qhi,
                                   float& qlo) {
  const float d2lo = fmaf(-2.0f, gx, ta.x + tb.x);
  const float d2hi = fmaf(-2.0f, gx, ta.y + tb.y);
  const float e2lo = fmaf(-2.0f, gy, ta.z + tb.z);
  const float e2hi = fmaf(-2.0f, gy, ta.w + tb.w);
  const float h = fmaxf(e2hi, 0.0f) * __builtin_amdgcn_rcpf(d2lo);
  const float l = fmaxf(e2lo, 0.0f) * __builtin_amdgcn_rcpf(d2hi);
  qhi = d2lo > 1e-30f ? h : 3.0e38f;
  qlo = d2hi > 1e-30f ? l : 0.0f;
  if (!(d2hi > 0.0f)) { qhi = 1.0f; qlo = 1.0f; }
}

// Bounds on q for one pair of a compact-cache screen, from its cached g,
// the image Gram entry and the row terms (c: the cache's constant, ic = 1/c).
// D^2 <= D2lo + 1.25 (width_i + width_j) (the bound the FP32 epilogue's d2hi
// also satisfies) and D2lo <= (1 + 2^-10 + 2^-20) c / g, or D2lo < c 2^-15
// when g is infinite, so
//   D2hi' = (1 + 2^-10 + 2^-18) fl(c / g) + 1.25 (1 + 2^-20) w + c 2^-15
// (w = the two widths' sum), formed with two FMAs, is an upper bound on D^2:
// the margins absorb the roundings of the division, of w and of both FMAs.
// q_hi = (E2hi / c) g while g is finite; an infinite g (identical or nearly
// identical points) gets the widest upper bound and the pair is re-examined.
__device__ inline void pair_bounds_compact(float g, float gy, const float4& ta, const float4& tb, float c,
                                           float ic, float& qhi, float& qlo) {
  const float e2lo = fmaf(-2.0f, gy, ta.z + tb.z);
  const float e2hi = fmaf(-2.0f, gy, ta.w + tb.w);
  const float w = (ta.y - ta.x) + (tb.y - tb.x);
  const float d2hi = fmaf(c / g, 0x1.00404p+0f, fmaf(w, 0x1.400014p+0f, c * 0x1p-15f));
  qhi = g < INFINITY ? (fmaxf(e2hi, 0.0f) * ic) * g : 3.0e38f;
  qlo = fmaxf(e2lo, 0.0f) * __builtin_amdgcn_rcpf(d2hi);
}

// Wave-wide integer minimum (all lanes receive it).  On the bits of FP32
// values it is the smallest value while all are positive, and a negative
// value's bits (or -0's) whenever one is present.
__device__ inline int32_t wave_min_i32(int32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const int32_t w = __shfl_xor(v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}

// A tile's point Gram (accumulators in the D layout) turned in place into the
// pairs' D2lo = (lo_i + lo_j) - 2 g, the value the FP32 epilogue bounds D^2
// from below with; what a compact cache block stores.
__device__ inline void gram_to_d2lo(f32x16 (&acc)[2][2], const float4* termA, const float4* termB) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1, li = lane & 31, lh = lane >> 5;
  const float b0 = termB[wc * 64 + li].x, b1 = termB[wc * 64 + 32 + li].x;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float a = termA[wr * 64 + x * 32 + (v >> 2) * 8 + lh * 4 + (v & 3)].x;
      acc[x][0][v] = fmaf(-2.0f, acc[x][0][v], a + b0);
      acc[x][1][v] = fmaf(-2.0f, acc[x][1][v], a + b1);
    }
}

// Wave-wide reductions (all lanes receive the result).
__device__ inline uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t w = (uint32_t)__shfl_xor((int)v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}
__device__ inline uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t w = (uint32_t)__shfl_xor((int)v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}
__device__ inline float wave_min_f32(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline float wave_max_f32(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// Sortable key of a non-negative FP32 value and a 6-bit pair code: the
// value's bits with the low 6 mantissa bits replaced by the code (the sign
// bit dropped, so -0 sorts as 0).  For keys k of values q:
// q <= key_hi_value(max k) and q >= key_lo_value(min k).
__device__ inline uint32_t pair_key(float q, int code) {
  return (__float_as_uint(q) & 0x7FFFFFC0u) | (uint32_t)code;
}
__device__ inline float key_hi_value(uint32_t k) { return __uint_as_float((k & 0xFFFFFFC0u) | 63u); }
__device__ inline float key_lo_value(uint32_t k) { return __uint_as_float(k & 0xFFFFFFC0u); }

// Epilogue of one 128 x 128 tile, shared by the screen kernels.  accX/accY
// hold the point and image Gram blocks of this wave in the D layout of the
// 32 x 32 MFMAs (lane l, register v -> row (v / 4) * 8 + (l / 32) * 4 + v % 4,
// column l % 32), which is the same for v_mfma_f32_32x32x2f32 and
// v_mfma_f32_32x32x16_bf16.  MODE 0 writes the tile record (after a
// block-wide barrier); MODE 1 appends the pairs reaching the thresholds.
// COMPACT: px is the tile's compact cache block (packed FP16 g values, see
// dcache_load) in place of the point Gram accX.
template <bool COMPACT, typename PX>
__device__ __attribute__((always_inline)) inline float point_side(const PX& px, int x, int y, int v) {
  if constexpr (COMPACT) return dcache_g(px, x, y, v);
  else return px[x][y][v];
}
// The part of one wave's 64 x 64 block: `wave` (0..3) is the block's place
// in the tile (rows (wave / 2) * 64, columns (wave % 2) * 64); MODE 0 leaves
// the block's record in red_*[.][wave], MODE 1 appends its pairs.  A kernel
// whose waves hold two such blocks calls it once per block.
template <int MODE, bool COMPACT = false, typename PX>
__device__ __attribute__((always_inline)) inline void wave_epilogue(const PX& accX, const f32x16 (&accY)[2][2],
                                     const float4* termA, const float4* termB, int I, int J,
                                     const PairsArgs& p, float thr_hi, float thr_lo, float (*red_v)[4],
                                     int (*red_i)[4], int (*red_j)[4], int wave) {
  const int lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 31, lh = lane >> 5;
  const int row0 = I * kTile, col0 = J * kTile;
  // D layout of v_mfma_f32_32x32x2f32: lane l, register v ->
  // row (v / 4) * 8 + (l / 32) * 4 + v % 4, column l % 32.
  // Edge tiles (diagonal, or past the last point) mask invalid pairs.
  const bool masked = !((I < J) && (col0 + kTile <= p.n));
  float best_hi = -1.0f, best_lo = 3.0e38f;
  int code_hi = -1, code_lo = -1, code_c = -1;
  const float stop_hi = p.stop_hi, stop_lo = p.stop_lo;
  const float4 tb0 = termB[wc * 64 + li], tb1 = termB[wc * 64 + 32 + li];
  const float dc = COMPACT ? *p.dscale : 1.0f, idc = 1.0f / dc;   // exact: a power of two
  // The pass over the thread's 64 pairs, compiled once with the edge mask and
  // once without (the mask is uniform per tile: no per-pair branch).
  auto scan = [&](auto maskc) __attribute__((always_inline)) {
    constexpr bool M = decltype(maskc)::value;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rl = wr * 64 + x * 32 + (v >> 2) * 8 + lh * 4 + (v & 3);
        const float4 ta = termA[rl];
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          float qhi, qlo;
          const float pv = point_side<COMPACT>(accX, x, y, v);
          if (COMPACT) pair_bounds_compact(pv, accY[x][y][v], ta, y ? tb1 : tb0, dc, idc, qhi, qlo);
          else pair_bounds(pv, accY[x][y][v], ta, y ? tb1 : tb0, qhi, qlo);
          bool certain = MODE == 0 && (qlo > stop_hi || qhi < stop_lo);
          if (M) {
            const int cl = wc * 64 + y * 32 + li;
            const bool valid = (I < J || rl < cl) && col0 + cl < p.n;
            if (!valid) { qhi = -1.0f; qlo = 3.0e38f; certain = false; }
          }
          if (MODE == 0) {
            const int code = (x * 2 + y) * 16 + v;
            if (qhi > best_hi) { best_hi = qhi; code_hi = code; }
            if (qlo < best_lo) { best_lo = qlo; code_lo = code; }
            if (certain) code_c = code;
            // Pin the running arg-extremes here: otherwise the compiler first
            // evaluates all 64 pairs (128 live values) and spills.
            asm volatile("" : "+v"(best_hi), "+v"(code_hi), "+v"(best_lo), "+v"(code_lo), "+v"(code_c));
          } else {
            if (qhi >= thr_hi || qlo <= thr_lo) {
              const uint32_t pos = atomicAdd(p.ncand, 1u);
              const int cl = wc * 64 + y * 32 + li;
              if (pos < p.cap) p.cand[pos] = make_int2(row0 + rl, col0 + cl);
            }
          }
        }
      }
  };
  auto decode = [&](int code, int& gi, int& gj) {
    if (code < 0) { gi = 0x7fffffff; gj = 0x7fffffff; return; }
    const int x = code >> 5, y = (code >> 4) & 1, v = code & 15;
    gi = row0 + wr * 64 + x * 32 + (v >> 2) * 8 + lh * 4 + (v & 3);
    gj = col0 + wc * 64 + y * 32 + li;
  };

  // MODE 0 fast pass: per pair only the rigorous upper bound
  // q+ = E2hi / D2lo (E2hi = (hi_i + hi_j) - 2 g_y, D2lo = (lo_i + lo_j) - 2 g_x),
  // kept as sortable keys (largest and smallest per lane), and the smallest
  // D2lo and E2hi.  The wave's record then takes
  //   q_hi = the largest q+ (rounded up),
  //   q_lo = the smallest q+ x (1 - W_E / E2hi_min) / (1 + W_D / D2lo_min) (rounded down),
  // where W_D, W_E >= 1.25 (width_i + width_j) bound D2hi - D2lo and
  // E2hi - E2lo over the wave's rows i and columns j (width = hi - lo of a
  // row term, which also covers the rounding of the epilogue's add and fma):
  // for every pair E2 >= E2hi - W_E and D2 <= D2lo + W_D, so
  // E2 / D2 >= q+ (1 - W_E / E2hi) / (1 + W_D / D2lo), and the factor grows
  // with E2hi and D2lo.  A wave whose smallest D2lo or E2hi is within 64
  // widths (so q_lo would lose more than about 3%), holds a pair with
  // D2lo <= 1e-30 (identical or nearly identical points) or a q+ near FP32
  // overflow takes the per-pair pass above instead.
  // COMPACT: per pair q+ = E2hi g / c (g >= c / D2lo), and since
  // D2lo <= (1 + 2^-10 + 2^-20) c / g, the same steps give the factor
  // (1 - W_E / E2hi_min) / (1 + 2^-10 + 2^-19 + W_D g_max / c); the wave
  // takes the per-pair pass when g_max is infinite or W_D g_max / c >= 1/64.
  // The keys hold E2hi g (c q+), scaled by 1/c (exactly) once per wave.
  // The running minima are kept as integers on the values' bits (positive
  // FP32 values order like their bits, and a negative value's bits, or -0's,
  // are below every positive one's), which spares the NaN handling of fminf.
  bool fast = false;
  if (MODE == 0) {
    uint32_t khi = 0u, klo = 0xFFFFFFFFu;
    int32_t dmin = 0x7F7FFFFF, emin = 0x7F7FFFFF;   // FP32 path: smallest D2lo; smallest E2hi
    uint32_t gmax = 0u;                              // COMPACT: largest g
    auto fscan = [&](auto maskc) __attribute__((always_inline)) {
      constexpr bool M = decltype(maskc)::value;
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int rl = wr * 64 + x * 32 + (v >> 2) * 8 + lh * 4 + (v & 3);
          const float4 ta = termA[rl];
#pragma unroll
          for (int y = 0; y < 2; ++y) {
            const float4 tb = y ? tb1 : tb0;
            const float e2hi = fmaf(-2.0f, accY[x][y][v], ta.w + tb.w);
            // dv: g (COMPACT) or D2lo
            const float pv = point_side<COMPACT>(accX, x, y, v);
            const float dv = COMPACT ? pv : fmaf(-2.0f, pv, ta.x + tb.x);
            const float q = COMPACT ? e2hi * dv : e2hi * __builtin_amdgcn_rcpf(dv);
            const uint32_t k = pair_key(q, (x * 2 + y) * 16 + v);
            const int32_t di = __float_as_int(dv), ei = __float_as_int(e2hi);
            bool valid = true;
            if (M) {
              const int cl = wc * 64 + y * 32 + li;
              valid = (I < J || rl < cl) && col0 + cl < p.n;
            }
            khi = valid && k > khi ? k : khi;
            klo = valid && k < klo ? k : klo;
            if (COMPACT) gmax = valid && (uint32_t)di > gmax ? (uint32_t)di : gmax;
            else dmin = valid && di < dmin ? di : dmin;
            emin = valid && ei < emin ? ei : emin;
            // pinned per pair, as in the per-pair pass (else the compiler
            // evaluates many pairs first and runs out of registers)
            asm volatile("" : "+v"(khi), "+v"(klo), "+v"(dmin), "+v"(emin), "+v"(gmax));
          }
        }
    };
    if (masked) fscan(std::integral_constant<bool, true>{});
    else fscan(std::integral_constant<bool, false>{});
    // widths of the wave's 64 rows and 64 columns, one of each per lane
    const float4 ra = termA[wr * 64 + lane], cb = termB[wc * 64 + lane];
    const float wDr = wave_max_f32(ra.y - ra.x), wEr = wave_max_f32(ra.w - ra.z);
    const float wDc = wave_max_f32(cb.y - cb.x), wEc = wave_max_f32(cb.w - cb.z);
    const uint32_t whi = wave_max_u32(khi), wlo = wave_min_u32(klo);
    const float we = __int_as_float(wave_min_i32(emin));
    const double WD = 1.25 * ((double)wDr + (double)wDc), WE = 1.25 * ((double)wEr + (double)wEc);
    // dterm = W_D / D2lo_min, or W_D g_max / c
    double dterm;
    bool dok;
    if constexpr (COMPACT) {
      const uint32_t gm = wave_max_u32(gmax);
      dok = gm < 0x7F800000u;
      dterm = WD * (double)__uint_as_float(gm) * (double)idc;
    } else {
      const float wd = __int_as_float(wave_min_i32(dmin));
      dok = wd > 1e-30f;
      dterm = WD / (double)wd;
    }
    const double rel = COMPACT ? 0x1p-10 + 0x1p-19 : 0.0, sc = (double)idc;
    // a wave without valid pairs (whi = 0, wlo = ~0) has no record to make
    const bool any = wlo != 0xFFFFFFFFu;
    fast = any && dok && dterm * 64.0 < 1.0 && (double)we > 64.0 * WE && whi < 0x7F000000u;
    if (fast) {
      float vhi = key_hi_value(whi);
      if (COMPACT) {   // the scaling by 1/c, rounded up
        const double h = (double)vhi * sc;
        vhi = (float)h;
        if ((double)vhi < h) vhi = __uint_as_float(__float_as_uint(vhi) + 1u);
      }
      const double f = (1.0 - WE / (double)we) / (1.0 + rel + dterm);
      const float vlo = (float)((double)key_lo_value(wlo) * sc * (1.0 - 0x1.0p-20) * f * (1.0 - 1e-7));
      // the lanes holding the wave's extreme keys (lowest lane among equal keys)
      const uint64_t bh = __ballot(khi == whi), bl = __ballot(klo == wlo);
      const int lhi = __ffsll((unsigned long long)bh) - 1, llo = __ffsll((unsigned long long)bl) - 1;
      int ih, jh, il, jl;
      decode((int)(khi & 63u), ih, jh);
      decode((int)(klo & 63u), il, jl);
      ih = __shfl(ih, lhi, 64); jh = __shfl(jh, lhi, 64);
      il = __shfl(il, llo, 64); jl = __shfl(jl, llo, 64);
      // early stop: the expansion winner's q >= its q+ x factor, the
      // contraction winner's q <= its q+
      if (p.stop && lane == 0) {
        const bool c_hi = (double)key_lo_value(whi) * sc * (1.0 - 0x1.0p-20) * f > (double)stop_hi;
        const bool c_lo = (double)key_hi_value(wlo) * sc < (double)stop_lo;
        if (c_hi || c_lo) {
          const uint32_t pos = atomicAdd(p.stop, 1u);
          if (pos < 8) p.stop_pairs[pos] = c_hi ? make_int2(ih, jh) : make_int2(il, jl);
        }
      }
      if (lane == 0) {
        red_v[0][wave] = vhi; red_i[0][wave] = ih; red_j[0][wave] = jh;
        red_v[1][wave] = vlo; red_i[1][wave] = il; red_j[1][wave] = jl;
      }
    } else if (!any && lane == 0) {
      red_v[0][wave] = -1.0f; red_i[0][wave] = 0x7fffffff; red_j[0][wave] = 0x7fffffff;
      red_v[1][wave] = 3.0e38f; red_i[1][wave] = 0x7fffffff; red_j[1][wave] = 0x7fffffff;
    }
    fast = fast || !any;
  }

  if (MODE == 1 || !fast) {
    if (masked) scan(std::integral_constant<bool, true>{});
    else scan(std::integral_constant<bool, false>{});
  }

  if (MODE == 0) {
    if (!fast) {
    int ih, jh, il, jl;
    if (p.stop && code_c >= 0) {   // rare: a pair certain to exceed the target
      decode(code_c, ih, jh);
      const uint32_t pos = atomicAdd(p.stop, 1u);
      if (pos < 8) p.stop_pairs[pos] = make_int2(ih, jh);
    }
    decode(code_hi, ih, jh);
    decode(code_lo, il, jl);
    wave_arg<true>(best_hi, ih, jh);
    wave_arg<false>(best_lo, il, jl);
    if (lane == 0) {
      red_v[0][wave] = best_hi; red_i[0][wave] = ih; red_j[0][wave] = jh;
      red_v[1][wave] = best_lo; red_i[1][wave] = il; red_j[1][wave] = jl;
    }
    }
  }
}

// MODE 0: the tile record from the four blocks' records, after a block-wide
// barrier.
__device__ __attribute__((always_inline)) inline void tile_record(int I, int J, const PairsArgs& p,
                                                                  float (*red_v)[4], int (*red_i)[4],
                                                                  int (*red_j)[4]) {
  {
    __syncthreads();
    if (threadIdx.x == 0) {
      float vh = red_v[0][0], vl = red_v[1][0];
      int ih0 = red_i[0][0], jh0 = red_j[0][0], il0 = red_i[1][0], jl0 = red_j[1][0];
      for (int w = 1; w < 4; ++w) {
        if (red_v[0][w] > vh || (red_v[0][w] == vh && idx_better(red_i[0][w], red_j[0][w], ih0, jh0))) {
          vh = red_v[0][w]; ih0 = red_i[0][w]; jh0 = red_j[0][w];
        }
        if (red_v[1][w] < vl || (red_v[1][w] == vl && idx_better(red_i[1][w], red_j[1][w], il0, jl0))) {
          vl = red_v[1][w]; il0 = red_i[1][w]; jl0 = red_j[1][w];
        }
      }
      // an invalid pair (code < 0 or masked) never wins against a valid one:
      // valid q_hi >= 0 > -1 and valid q_lo <= 3e38.
      const bool none_hi = ih0 == 0x7fffffff || vh < 0.0f;
      const bool none_lo = il0 == 0x7fffffff || vl >= 3.0e38f;
      TileRec rec;
      rec.qhi = vh; rec.qlo = vl;
      rec.ihi = none_hi ? -1 : ih0; rec.jhi = none_hi ? -1 : jh0;
      rec.ilo = none_lo ? -1 : il0; rec.jlo = none_lo ? -1 : jl0;
      rec.pad0 = 0; rec.pad1 = 0;
      const int64_t t = (int64_t)I * p.NT - (int64_t)I * (I - 1) / 2 + (J - I);
      p.recs[t] = rec;
    }
  }
}

template <int MODE, bool COMPACT = false, typename PX>
__device__ __attribute__((always_inline)) inline void tile_epilogue(const PX& accX, const f32x16 (&accY)[2][2],
                                     const float4* termA, const float4* termB, int I, int J,
                                     const PairsArgs& p, float thr_hi, float thr_lo, float (*red_v)[4],
                                     int (*red_i)[4], int (*red_j)[4]) {
  wave_epilogue<MODE, COMPACT>(accX, accY, termA, termB, I, J, p, thr_hi, thr_lo, red_v, red_i, red_j,
                               (int)(threadIdx.x >> 6));
  if (MODE == 0) tile_record(I, J, p, red_v, red_i, red_j);
}

}  // namespace adg
