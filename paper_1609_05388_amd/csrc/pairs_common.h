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
__device__ inline void gcache_store(float* cache, int64_t tile, const f32x16 (&acc)[2][2]) {
  float4* g = reinterpret_cast<float4*>(cache) + tile * 4096 + threadIdx.x;
#pragma unroll
  for (int k4 = 0; k4 < 16; ++k4) {
    const f32x16& a = acc[k4 >> 3][(k4 >> 2) & 1];
    const int v = (k4 & 3) * 4;
    g[k4 * 256] = make_float4(a[v], a[v + 1], a[v + 2], a[v + 3]);
  }
}
__device__ inline void gcache_load(const float* cache, int64_t tile, f32x16 (&acc)[2][2]) {
  const float4* g = reinterpret_cast<const float4*>(cache) + tile * 4096 + threadIdx.x;
#pragma unroll
  for (int k4 = 0; k4 < 16; ++k4) {
    const float4 t = g[k4 * 256];
    f32x16& a = acc[k4 >> 3][(k4 >> 2) & 1];
    const int v = (k4 & 3) * 4;
    a[v] = t.x; a[v + 1] = t.y; a[v + 2] = t.z; a[v + 3] = t.w;
  }
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

// Epilogue of one 128 x 128 tile, shared by the screen kernels.  accX/accY
// hold the point and image Gram blocks of this wave in the D layout of the
// 32 x 32 MFMAs (lane l, register v -> row (v / 4) * 8 + (l / 32) * 4 + v % 4,
// column l % 32), which is the same for v_mfma_f32_32x32x2f32 and
// v_mfma_f32_32x32x16_bf16.  MODE 0 writes the tile record (after a
// block-wide barrier); MODE 1 appends the pairs reaching the thresholds.
template <int MODE>
__device__ inline void tile_epilogue(const f32x16 (&accX)[2][2], const f32x16 (&accY)[2][2],
                                     const float4* termA, const float4* termB, int I, int J,
                                     const PairsArgs& p, float thr_hi, float thr_lo, float (*red_v)[4],
                                     int (*red_i)[4], int (*red_j)[4]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
          pair_bounds(accX[x][y][v], accY[x][y][v], ta, y ? tb1 : tb0, qhi, qlo);
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
  if (masked) scan(std::integral_constant<bool, true>{});
  else scan(std::integral_constant<bool, false>{});

  if (MODE == 0) {
    auto decode = [&](int code, int& gi, int& gj) {
      if (code < 0) { gi = 0x7fffffff; gj = 0x7fffffff; return; }
      const int x = code >> 5, y = (code >> 4) & 1, v = code & 15;
      gi = row0 + wr * 64 + x * 32 + (v >> 2) * 8 + lh * 4 + (v & 3);
      gj = col0 + wc * 64 + y * 32 + li;
    };
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
    __syncthreads();
    if (tid == 0) {
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
    return;
  }
}

}  // namespace adg
