// Step a7: the all-pairs screen of the eq. (3) certificate.
//
// For every unordered pair i < j the distortion of eq. (2) is
// | sqrt(q) - 1 | with q = E^2 / D^2, D^2 = ||x_i - x_j||^2 and
// E^2 = ||y_i - y_j||^2.  With centred FP32 rows a (points) and b (images),
//   D^2 = |a_i|^2 + |a_j|^2 - 2 a_i.a_j,   E^2 = |b_i|^2 + |b_j|^2 - 2 b_i.b_j,
// so one 128 x 128 tile of pairs is two Gram blocks: the a-Gram over the d
// point coordinates and the b-Gram over the r image coordinates, both on
// v_mfma_f32_32x32x2f32.  The epilogue turns them into rigorous bounds
//   D^2_lo/hi = (lo_i + lo_j) - 2 g_a,  (hi_i + hi_j) - 2 g_a   (same for E^2)
// where the per-row terms lo/hi carry the FP32 rounding of centring, norms,
// the MFMA dot product and the epilogue arithmetic, and
//   q_hi = E^2_hi / D^2_lo >= q,   q_lo = E^2_lo / D^2_hi <= q.
// A pair's distortion is at most max(sqrt(q_hi) - 1, 1 - sqrt(q_lo)).
//
// MODE 0 (screen): one tile per workgroup; the tile's largest q_hi and
//   smallest q_lo with their pairs go to a tile record.
// MODE 1 (emit): workgroups walk a list of flagged tiles and append every
//   pair whose bounds reach the thresholds (q_hi >= thr_hi or q_lo <= thr_lo)
//   to a candidate list for exact FP64 re-evaluation.
//
// Layout: rows padded to a multiple of 128 (zero rows), columns to a multiple
// of 16 (zero columns).  Tile order: the upper triangle of 128 x 128 tiles is
// cut into 8 x 8 super-tiles (SI <= SJ, row-major); a slot s names tile
// (8 SI + (s mod 64) / 8, 8 SJ + s mod 8) of super-tile s / 64 (slots below
// the diagonal or past the last tile exit at once).  Workgroup b runs on XCD
// b mod 8, so slot = (b mod 8) * (G / 8) + b / 8 gives every XCD a contiguous
// run of super-tiles: the ~64 workgroups resident on an XCD work on one
// super-tile and share its 8 row panels and 8 column panels in that XCD's L2.
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "pairs_common.h"

namespace adg {

constexpr int PT = kTile;   // 128
constexpr int PK = kChunk;  // 16
constexpr int PLD = 16;     // LDS row stride in floats (no padding; see lds_at)

// LDS position of float4 number q (0..3) of row `row` in a chunk buffer: the
// float4s of a row are XOR-swizzled with bits 2-3 of the row, so that both
// the staging writes (4 rows x 4 float4s per 16 lanes) and the MFMA operand
// reads (16 rows x 1 float4 per 16 lanes) hit 16 distinct 4-bank groups.
__device__ inline int lds_at(int row, int q) { return row * PLD + ((q ^ (row >> 2)) & 3) * 4; }


// LOADED (MODE 0 only): the point Gram comes from the cache; the kernel runs
// the image chunks only and loads the point-Gram accumulators after them, so
// far fewer registers are live in its loop and three workgroups fit a CU.
template <int MODE, bool LOADED>
__global__ __launch_bounds__(256, LOADED ? 3 : 2) void k_pairs_f32(PairsArgs p) {
  __shared__ __attribute__((aligned(16))) float As[2][PT * PLD];
  __shared__ __attribute__((aligned(16))) float Bs[2][PT * PLD];
  __shared__ float4 termA[PT], termB[PT];
  __shared__ float red_v[2][4];
  __shared__ int red_i[2][4], red_j[2][4];
  __shared__ uint32_t s_stop;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 31, lh = lane >> 5;
  const int total = p.nchx + p.nchy;

  int I, J;
  uint32_t u = blockIdx.x, u_end = 1;
  float thr_hi = 0.f, thr_lo = 0.f;
  if (MODE == 0) {
    const uint32_t G = gridDim.x;
    const int64_t slot = (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
    if (slot >= p.nslots) return;
    const TilePos tp = slot_tile(slot, p.NT, p.NS);
    if (tp.I < 0) return;
    I = (int)tp.I;
    J = (int)tp.J;
  } else {
    u_end = p.cd->n_flagged;
    thr_hi = p.cd->thr_hi;
    thr_lo = p.cd->thr_lo;
    if (u >= u_end) return;
  }

  for (;;) {
    if (MODE == 1) {
      const TilePos tp = tri_tile_p(p.list[u], p.NT);
      I = (int)tp.I;
      J = (int)tp.J;
    }
    const int row0 = I * PT, col0 = J * PT;
    // no tile records: the launch only fills the point-Gram cache
    const bool store_only = MODE == 0 && p.recs == nullptr;
    // The tile's first chunk, its row terms and (MODE 0) the early-stop flag
    // are all requested before any of them is waited for: the first chunk's
    // loads, then these two, whose LDS stores follow the first stash.
    // Thread t < 128 holds the terms of row t of the tile's rows, t >= 128
    // of its columns; the flag is shared through LDS at the first barrier
    // (a uniform exit).
    float4 side_t = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    uint32_t side_s = 0u;
    auto load_side = [&]() __attribute__((always_inline)) {
      if (!store_only) {
        const int row = tid < PT ? row0 + tid : col0 + tid - PT;
        const float2 a = p.tx[row], b = p.ty[row];
        side_t = make_float4(a.x, a.y, b.x, b.y);
      }
      if (MODE == 0 && tid == 0 && p.stop)
        side_s = __hip_atomic_load(p.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    auto store_side = [&]() __attribute__((always_inline)) {
      if (!store_only) {
        if (tid < PT) termA[tid] = side_t;
        else termB[tid - PT] = side_t;
      }
      if (MODE == 0 && tid == 0) s_stop = side_s;
    };

    // ---------------------------------------------------------- Gram phase
    f32x16 accX[2][2], accY[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        accX[a][b] = (f32x16){0};
        accY[a][b] = (f32x16){0};
      }

    const int lr = tid >> 2, lc = (tid & 3) * 4;
    const float* xa = p.X + (size_t)(row0 + lr) * p.ldx + lc;
    const float* xb = p.X + (size_t)(col0 + lr) * p.ldx + lc;
    const float* ya = p.Y + (size_t)(row0 + lr) * p.ldy + lc;
    const float* yb = p.Y + (size_t)(col0 + lr) * p.ldy + lc;
    const size_t x64 = (size_t)64 * p.ldx, y64 = (size_t)64 * p.ldy;
    // two register sets of staging loads (the second for the pipelined image
    // loop of the LOADED kernel)
    float4 ga0, ga1, gb0, gb1, ha0, ha1, hb0, hb1;
    auto fetch_into = [&](float4& a0, float4& a1, float4& b0, float4& b1, int c) __attribute__((always_inline)) {
      if (c < p.nchx) {
        const int cb = c * PK;
        a0 = *reinterpret_cast<const float4*>(xa + cb);
        a1 = *reinterpret_cast<const float4*>(xa + x64 + cb);
        b0 = *reinterpret_cast<const float4*>(xb + cb);
        b1 = *reinterpret_cast<const float4*>(xb + x64 + cb);
      } else {
        const int cb = (c - p.nchx) * PK;
        a0 = *reinterpret_cast<const float4*>(ya + cb);
        a1 = *reinterpret_cast<const float4*>(ya + y64 + cb);
        b0 = *reinterpret_cast<const float4*>(yb + cb);
        b1 = *reinterpret_cast<const float4*>(yb + y64 + cb);
      }
    };
    auto stash_from = [&](const float4& a0, const float4& a1, const float4& b0, const float4& b1, int buf)
        __attribute__((always_inline)) {
      *reinterpret_cast<float4*>(&As[buf][lds_at(lr, lc >> 2)]) = a0;
      *reinterpret_cast<float4*>(&As[buf][lds_at(lr + 64, lc >> 2)]) = a1;
      *reinterpret_cast<float4*>(&Bs[buf][lds_at(lr, lc >> 2)]) = b0;
      *reinterpret_cast<float4*>(&Bs[buf][lds_at(lr + 64, lc >> 2)]) = b1;
    };
    auto fetch = [&](int c) __attribute__((always_inline)) { fetch_into(ga0, ga1, gb0, gb1, c); };
    auto stash = [&](int buf) __attribute__((always_inline)) { stash_from(ga0, ga1, gb0, gb1, buf); };
    auto fetch2 = [&](int c) __attribute__((always_inline)) { fetch_into(ha0, ha1, hb0, hb1, c); };
    auto stash2 = [&](int buf) __attribute__((always_inline)) { stash_from(ha0, ha1, hb0, hb1, buf); };
    // MFMA step kk sums columns kk (lanes 0-31) and 8 + kk (lanes 32-63) of
    // the chunk; the same permutation is used for both operands.
    auto mma = [&](f32x16 (&acc)[2][2], int buf) __attribute__((always_inline)) {
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        float4 a4[2], b4[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          a4[x] = *reinterpret_cast<const float4*>(&As[buf][lds_at(wr * 64 + x * 32 + li, lh * 2 + half)]);
          b4[x] = *reinterpret_cast<const float4*>(&Bs[buf][lds_at(wc * 64 + x * 32 + li, lh * 2 + half)]);
        }
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
              acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[x][kk], b4[y][kk], acc[x][y], 0, 0, 0);
      }
    };

    // Two loops with fixed accumulators (one selected per chunk would make
    // the compiler copy the other set); the prefetch runs across the seam.
    // With a loaded point Gram the pipeline starts at the first image chunk.
    const int64_t tix = (int64_t)I * p.NT - (int64_t)I * (I - 1) / 2 + (J - I);
    if (LOADED) {
      // image chunk k (0 <= k < nk) sits in LDS buffer k & 1 and, while in
      // flight, in register set k & 1: the next two chunks load while one
      // is multiplied
      const int nk = p.nchy, cy = p.nchx;
      fetch(cy);
      load_side();   // before the second chunk: the first barrier waits for these
      if (nk > 1) fetch2(cy + 1);
      stash(0);
      store_side();
      __syncthreads();
      if (MODE == 0 && s_stop != 0u) return;
      int k = 0;
      for (; k + 2 < nk; k += 2) {
        fetch(cy + k + 2);
        mma(accY, 0);
        stash2(1);
        __syncthreads();
        if (k + 3 < nk) fetch2(cy + k + 3);
        mma(accY, 1);
        stash(0);
        __syncthreads();
      }
      // the last one or two chunks; then the cached point Gram, where its
      // accumulators become live (issued before these MFMAs it would wait
      // behind the staging loads, which the vector-memory counter completes
      // in issue order, and hold registers through the loop)
      mma(accY, 0);
      if (k + 1 < nk) {
        stash2(1);
        __syncthreads();
        mma(accY, 1);
      }
      gcache_load(p.gcache, tix, accX);
    } else {
      fetch(0);
      load_side();
      stash(0);
      store_side();
      __syncthreads();
      if (MODE == 0 && s_stop != 0u) return;
      for (int c = 0; c < p.nchx; ++c) {
        const int buf = c & 1;
        if (c + 1 < total) fetch(c + 1);
        mma(accX, buf);
        if (c + 1 < total) stash(buf ^ 1);
        __syncthreads();
      }
      for (int c = p.nchx; c < total; ++c) {
        const int buf = c & 1;
        if (c + 1 < total) fetch(c + 1);
        mma(accY, buf);
        if (c + 1 < total) stash(buf ^ 1);
        __syncthreads();
      }
    }
    // stores after the image loop (earlier they would hold up its chunk
    // loads, which the vector-memory counter completes in issue order)
    if (!LOADED && MODE == 0 && p.gmode == 1) gcache_store(p.gcache, tix, accX);
    if (store_only) return;

    tile_epilogue<MODE>(accX, accY, termA, termB, I, J, p, thr_hi, thr_lo, red_v, red_i, red_j);
    if (MODE == 0) return;
    u += gridDim.x;
    if (u >= u_end) return;
    __syncthreads();  // LDS terms / buffers are rewritten by the next tile
  }
}

hipError_t launch_pairs_screen(const PairsView& v, TileRec* recs, float* gcache, int gmode, const ScreenStop* stop,
                               hipStream_t st) {
  const int NS = (v.NT + 7) / 8;
  const int64_t nslots = (int64_t)NS * (NS + 1) / 2 * 64;
  PairsArgs a{v.X, v.ldx, v.ldx / PK, v.Y, v.ldy, v.ldy / PK, v.tx, v.ty, v.n, v.NT, v.ntiles,
              NS, nslots, recs, nullptr, nullptr, nullptr, 0u, nullptr, gcache, gcache ? gmode : 0,
              nullptr, nullptr, 3.0e38f, -1.0f};
  if (stop) {
    a.stop = stop->count; a.stop_pairs = stop->pairs; a.stop_hi = stop->q_hi; a.stop_lo = stop->q_lo;
  }
  const int64_t G = round_up(nslots, 8);
  if (a.gmode == 2) k_pairs_f32<0, true><<<(unsigned)G, 256, 0, st>>>(a);
  else k_pairs_f32<0, false><<<(unsigned)G, 256, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_pairs_gram_fill(const PairsView& v, float* gcache, hipStream_t st) {
  const int NS = (v.NT + 7) / 8;
  const int64_t nslots = (int64_t)NS * (NS + 1) / 2 * 64;
  PairsArgs a{v.X, v.ldx, v.ldx / PK, v.X, 0, 0, v.tx, v.tx, v.n, v.NT, v.ntiles,
              NS, nslots, nullptr, nullptr, nullptr, nullptr, 0u, nullptr, gcache, 1,
              nullptr, nullptr, 3.0e38f, -1.0f};
  k_pairs_f32<0, false><<<(unsigned)round_up(nslots, 8), 256, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_pairs_emit(const PairsView& v, const uint32_t* list, const CertDev* cd, int2* cand,
                             uint32_t cap, uint32_t* ncand, int grid, hipStream_t st) {
  PairsArgs a{v.X, v.ldx, v.ldx / PK, v.Y, v.ldy, v.ldy / PK, v.tx, v.ty, v.n, v.NT, v.ntiles,
              0, 0, nullptr, list, cd, cand, cap, ncand, nullptr, 0, nullptr, nullptr, 3.0e38f, -1.0f};
  k_pairs_f32<1, false><<<(unsigned)grid, 256, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace adg
