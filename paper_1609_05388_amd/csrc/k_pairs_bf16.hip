// Step a10 (precision form): the all-pairs screen with BF16 split-precision
// Grams.
//
// Every centred FP32 coordinate x is split as x = hi + lo + e with
// hi = bf16(x), lo = bf16(x - hi) (x - hi is exact in FP32) and
// |e| <= 2^-16 |x|.  A dot product is formed from three BF16 products,
//   x.y ~= hi_x.hi_y + hi_x.lo_y + lo_x.hi_y,
// on v_mfma_f32_32x32x16_bf16 with FP32 accumulation.  The dropped terms are
// at most 3.01 * 2^-16 sum |x_k||y_k| and the FP32 accumulation of 3K
// products at most gamma_3K * 1.012 sum |x_k||y_k|; the row terms carry these
// in place of the FP32 Gram's gamma_K, so the epilogue's bounds stay rigorous
// and the FP64 rescoring keeps the certificate exact.
//
// Operand layout in HBM: per row, per 16-column chunk, 16 hi values then 16
// lo values (64 bytes), so one chunk of one row is one contiguous 64-byte
// segment.  LDS rows are those 64 bytes, unpadded and XOR-swizzled by
// 16-byte segment (wide_at), free of bank conflicts for both the staging
// stores and the operand reads.  A 128 x 128 pair tile per workgroup of four
// waves (64 x 64 each, 2 x 2 MFMA blocks), 16-column chunks (one MFMA k-step)
// double buffered in LDS with the next chunks prefetched into registers; a
// workgroup needs 36 KB of LDS.
#include "common.h"
#include "kernels.h"
#include "pairs_common.h"

namespace adg {

constexpr int BK = 16;               // columns per chunk (one MFMA k-step)
constexpr int SEGS = BK / 4;         // 16-byte segments per row and chunk (hi 0-1, lo 2-3)
constexpr int SROWS = 256 / SEGS;    // rows one staging pass of 256 threads covers
constexpr int SPASS = kTile / SROWS; // staging passes per 128 rows
// LDS rows of one chunk are 64 bytes, unpadded: segment s of row r sits in
// slot s ^ ((r >> 2) & 3).  Sixteen consecutive rows (the 16-byte operand
// reads of 16 lanes) then cover all 64 banks, and so do four consecutive rows'
// four segments (the staging stores of 16 lanes).
constexpr int WROW = 4 * BK;
__device__ inline int wide_at(int row, int seg) { return row * WROW + ((seg ^ ((row >> 2) & 3)) << 4); }

// Split centred FP32 rows (n_pad x lds) into the chunk-interleaved BF16 hi/lo
// layout (n_pad rows of ldb * 2 bf16, ldb = columns rounded up to 32).
__global__ void k_split_bf16(const float* __restrict__ src, int64_t n_pad, int64_t m, int64_t lds,
                             int64_t ldb, __bf16* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n_pad * ldb) return;
  const int64_t row = e / ldb, col = e % ldb;
  const float x = col < m ? src[row * lds + col] : 0.0f;
  const __bf16 hi = (__bf16)x;
  const __bf16 lo = (__bf16)(x - (float)hi);
  const int64_t base = row * 2 * ldb + (col / BK) * (2 * BK) + (col % BK);
  dst[base] = hi;
  dst[base + BK] = lo;
}

struct PairsArgsB {
  const __bf16* X; int ldx; int nchx;  // hi/lo points, row stride 2 * ldx bf16, ldx = 16 * nchx
  const __bf16* Y; int ldy; int nchy;  // hi/lo images
  PairsArgs p;                         // row terms, sizes, outputs (X/Y fields unused)
};

// The screen with both Grams (no cache).  The screens of a fit with the
// compact cache are k_pairs_bf16x3_wide below, the cache's fill
// k_pairs_bf16x3_fill_quad.
template <int MODE>
__global__ __launch_bounds__(256, 2) void k_pairs_bf16x3(PairsArgsB b) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  unsigned char* As = lds_raw;                          // [2][128][WROW]
  unsigned char* Bs = lds_raw + 2 * kTile * WROW;       // [2][128][WROW]
  float4* termA = reinterpret_cast<float4*>(lds_raw + 4 * kTile * WROW);
  float4* termB = termA + kTile;
  float (*red_v)[4] = reinterpret_cast<float (*)[4]>(termB + kTile);
  int (*red_i)[4] = reinterpret_cast<int (*)[4]>(reinterpret_cast<float*>(red_v) + 8);
  int (*red_j)[4] = reinterpret_cast<int (*)[4]>(reinterpret_cast<int*>(red_i) + 8);
  // Copy the argument struct into locals: a reference into the by-value kernel
  // argument would make the compiler place a private copy in scratch memory.
  const PairsArgs p = b.p;
  const __bf16* const Xg = b.X;
  const __bf16* const Yg = b.Y;
  const int ldx = b.ldx, ldy = b.ldy, nchx = b.nchx, nchy = b.nchy;
  __shared__ uint32_t s_stop;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 31, lh = lane >> 5;
  const int total = nchx + nchy;

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
    const int row0 = I * kTile, col0 = J * kTile;
    // The tile's first chunks, its row terms and (MODE 0) the early-stop
    // flag are all requested before any of them is waited for: the first
    // chunk's loads, then these two, whose LDS stores follow the first stash.
    // Thread t < 128 holds the terms of row t of the tile's rows, t >= 128
    // of its columns; the flag is shared through LDS at the first barrier
    // (a uniform exit).
    auto load_side = [&](float4& tr, uint32_t& sv) __attribute__((always_inline)) {
      const int row = tid < kTile ? row0 + tid : col0 + tid - kTile;
      const float2 a = p.tx[row], c = p.ty[row];
      tr = make_float4(a.x, a.y, c.x, c.y);
      sv = MODE == 0 && tid == 0 && p.stop ? __hip_atomic_load(p.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                           : 0u;
    };
    auto store_side = [&](const float4& tr, uint32_t sv) __attribute__((always_inline)) {
      if (tid < kTile) termA[tid] = tr;
      else termB[tid - kTile] = tr;
      if (MODE == 0 && tid == 0) s_stop = sv;
    };
    float4 side_t;
    uint32_t side_s;

    f32x16 accX[2][2], accY[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        accX[x][y] = (f32x16){0};
        accY[x][y] = (f32x16){0};
      }

    // staging: thread t loads 16-byte segment (t % 8) of rows t / 8 + 32 m
    const int seg = tid % SEGS, lr = tid / SEGS;
    const size_t xstride = (size_t)2 * ldx, ystride = (size_t)2 * ldy;  // bf16 per row
    const __bf16* xa = Xg + (size_t)(row0 + lr) * xstride + seg * 8;
    const __bf16* xb = Xg + (size_t)(col0 + lr) * xstride + seg * 8;
    const __bf16* ya = Yg + (size_t)(row0 + lr) * ystride + seg * 8;
    const __bf16* yb = Yg + (size_t)(col0 + lr) * ystride + seg * 8;
    struct Stage {
      u32x4 a[SPASS], b[SPASS];
    };
    auto fetch_into = [&](Stage& g, int c) __attribute__((always_inline)) {
      if (c < nchx) {
        const size_t off = (size_t)c * 2 * BK;
#pragma unroll
        for (int m = 0; m < SPASS; ++m) {
          g.a[m] = *reinterpret_cast<const u32x4*>(xa + off + (size_t)SROWS * m * xstride);
          g.b[m] = *reinterpret_cast<const u32x4*>(xb + off + (size_t)SROWS * m * xstride);
        }
      } else {
        const size_t off = (size_t)(c - nchx) * 2 * BK;
#pragma unroll
        for (int m = 0; m < SPASS; ++m) {
          g.a[m] = *reinterpret_cast<const u32x4*>(ya + off + (size_t)SROWS * m * ystride);
          g.b[m] = *reinterpret_cast<const u32x4*>(yb + off + (size_t)SROWS * m * ystride);
        }
      }
    };
    auto stash_from = [&](const Stage& g, int buf) __attribute__((always_inline)) {
#pragma unroll
      for (int m = 0; m < SPASS; ++m) {
        *reinterpret_cast<u32x4*>(As + (size_t)buf * kTile * WROW + wide_at(lr + SROWS * m, seg)) = g.a[m];
        *reinterpret_cast<u32x4*>(Bs + (size_t)buf * kTile * WROW + wide_at(lr + SROWS * m, seg)) = g.b[m];
      }
    };
    Stage g0;
    auto fetch = [&](int c) __attribute__((always_inline)) { fetch_into(g0, c); };
    auto stash = [&](int buf) __attribute__((always_inline)) { stash_from(g0, buf); };
    // one k-step: lanes 0-31 take columns 0-7 (segment 0: hi, 2: lo), lanes
    // 32-63 columns 8-15 (segments 1 and 3).
    auto mma = [&](f32x16 (&acc)[2][2], int buf) __attribute__((always_inline)) {
      const unsigned char* A0 = As + (size_t)buf * kTile * WROW;
      const unsigned char* B0 = Bs + (size_t)buf * kTile * WROW;
      {
        bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          const int ra = wr * 64 + x * 32 + li, rb = wc * 64 + x * 32 + li;
          ah[x] = *reinterpret_cast<const bf16x8*>(A0 + wide_at(ra, lh));
          al[x] = *reinterpret_cast<const bf16x8*>(A0 + wide_at(ra, 2 + lh));
          bh[x] = *reinterpret_cast<const bf16x8*>(B0 + wide_at(rb, lh));
          bl[x] = *reinterpret_cast<const bf16x8*>(B0 + wide_at(rb, 2 + lh));
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[x], bh[y], acc[x][y], 0, 0, 0);
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[x], bl[y], acc[x][y], 0, 0, 0);
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[x], bh[y], acc[x][y], 0, 0, 0);
      }
    };

    {
      fetch(0);
      load_side(side_t, side_s);
      stash(0);
      store_side(side_t, side_s);
      __syncthreads();
      if (MODE == 0 && s_stop != 0u) return;
      for (int c = 0; c < nchx; ++c) {
        const int buf = c & 1;
        if (c + 1 < total) fetch(c + 1);
        mma(accX, buf);
        if (c + 1 < total) stash(buf ^ 1);
        __syncthreads();
      }
      for (int c = nchx; c < total; ++c) {
        const int buf = c & 1;
        if (c + 1 < total) fetch(c + 1);
        mma(accY, buf);
        if (c + 1 < total) stash(buf ^ 1);
        __syncthreads();
      }
    }
    tile_epilogue<MODE>(accX, accY, termA, termB, I, J, p, thr_hi, thr_lo, red_v, red_i, red_j);
    if (MODE == 0) return;
    u += gridDim.x;
    if (u >= u_end) return;
    __syncthreads();
  }
}

// The screen of a fit with the compact cache, with wider waves: two waves
// per 128 x 128 tile, wave w holding columns 64 w .. 64 w + 63 of all 128
// rows as 4 x 2 blocks of 32 x 32 (the blocks of two 64 x 64 waves of the
// other kernels, whose epilogue and cache layout it keeps).  Per chunk a
// wave runs 24 MFMAs between barriers (the four-wave kernel 12) and reads
// 12 KB of operands from LDS for them (16 KB for two waves' worth); 36 KB of
// LDS per workgroup.

__global__ __launch_bounds__(128, 2) void k_pairs_bf16x3_wide(PairsArgsB b) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  unsigned char* As = lds_raw;                          // [2][128][WROW]
  unsigned char* Bs = lds_raw + 2 * kTile * WROW;       // [2][128][WROW]
  float4* termA = reinterpret_cast<float4*>(lds_raw + 4 * kTile * WROW);
  float4* termB = termA + kTile;
  float (*red_v)[4] = reinterpret_cast<float (*)[4]>(termB + kTile);
  int (*red_i)[4] = reinterpret_cast<int (*)[4]>(reinterpret_cast<float*>(red_v) + 8);
  int (*red_j)[4] = reinterpret_cast<int (*)[4]>(reinterpret_cast<int*>(red_i) + 8);
  const PairsArgs p = b.p;
  const __bf16* const Yg = b.Y;
  const int ldy = b.ldy, nk = b.nchy;
  __shared__ uint32_t s_stop;
  const int tid = threadIdx.x, lane = tid & 63, wc = tid >> 6;
  const int li = lane & 31, lh = lane >> 5;

  const uint32_t G = gridDim.x;
  const int64_t slot = (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  if (slot >= p.nslots) return;
  const TilePos tp = slot_tile(slot, p.NT, p.NS);
  if (tp.I < 0) return;
  const int I = (int)tp.I, J = (int)tp.J;
  const int row0 = I * kTile, col0 = J * kTile;

  // staging: thread t loads segment t % 4 of rows t / 4 + 32 m (m = 0..3)
  const int seg = tid & 3, lr = tid >> 2;
  const size_t ystride = (size_t)2 * ldy;
  const __bf16* ya = Yg + (size_t)(row0 + lr) * ystride + seg * 8;
  const __bf16* yb = Yg + (size_t)(col0 + lr) * ystride + seg * 8;
  auto fetch_into = [&](u32x4 (&ra)[4], u32x4 (&rb)[4], int c) __attribute__((always_inline)) {
    const size_t off = (size_t)c * 2 * BK;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      ra[m] = *reinterpret_cast<const u32x4*>(ya + off + (size_t)32 * m * ystride);
      rb[m] = *reinterpret_cast<const u32x4*>(yb + off + (size_t)32 * m * ystride);
    }
  };
  auto stash_from = [&](const u32x4 (&ra)[4], const u32x4 (&rb)[4], int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      *reinterpret_cast<u32x4*>(As + (size_t)buf * kTile * WROW + wide_at(lr + 32 * m, seg)) = ra[m];
      *reinterpret_cast<u32x4*>(Bs + (size_t)buf * kTile * WROW + wide_at(lr + 32 * m, seg)) = rb[m];
    }
  };
  // one k-step: lanes 0-31 take columns 0-7 (segment 0: hi, 2: lo), lanes
  // 32-63 columns 8-15 (segments 1 and 3)
  f32x16 acc[2][2][2];   // [sub][x][y]: rows 64 sub + 32 x, columns 64 wc + 32 y
  auto mma = [&](int buf) __attribute__((always_inline)) {
    const unsigned char* A0 = As + (size_t)buf * kTile * WROW;
    const unsigned char* B0 = Bs + (size_t)buf * kTile * WROW;
    bf16x8 bh[2], bl[2];
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int r = wc * 64 + y * 32 + li;
      bh[y] = *reinterpret_cast<const bf16x8*>(B0 + wide_at(r, lh));
      bl[y] = *reinterpret_cast<const bf16x8*>(B0 + wide_at(r, 2 + lh));
    }
    // the two 64-row halves one after the other (half the A operands live)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      bf16x8 ah[2], al[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const int r = a * 64 + x * 32 + li;
        ah[x] = *reinterpret_cast<const bf16x8*>(A0 + wide_at(r, lh));
        al[x] = *reinterpret_cast<const bf16x8*>(A0 + wide_at(r, 2 + lh));
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[a][x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[x], bh[y], acc[a][x][y], 0, 0, 0);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[a][x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[x], bl[y], acc[a][x][y], 0, 0, 0);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[a][x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[x], bh[y], acc[a][x][y], 0, 0, 0);
    }
  };
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[a][x][y] = (f32x16){0};

  // the first chunk, then the row terms (thread t: row t of the tile's rows
  // and of its columns) and the early-stop flag, then the second chunk;
  // the first barrier waits for all but the second chunk
  u32x4 g0a[4], g0b[4], g1a[4], g1b[4];
  fetch_into(g0a, g0b, 0);
  const float2 ax = p.tx[row0 + tid], ay = p.ty[row0 + tid];
  const float2 bx = p.tx[col0 + tid], by = p.ty[col0 + tid];
  const uint32_t sv = tid == 0 && p.stop ? __hip_atomic_load(p.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                         : 0u;
  if (nk > 1) fetch_into(g1a, g1b, 1);
  stash_from(g0a, g0b, 0);
  termA[tid] = make_float4(ax.x, ax.y, ay.x, ay.y);
  termB[tid] = make_float4(bx.x, bx.y, by.x, by.y);
  if (tid == 0) s_stop = sv;
  __syncthreads();
  if (s_stop != 0u) return;
  int k = 0;
  for (; k + 2 < nk; k += 2) {
    fetch_into(g0a, g0b, k + 2);
    mma(0);
    stash_from(g1a, g1b, 1);
    __syncthreads();
    if (k + 3 < nk) fetch_into(g1a, g1b, k + 3);
    mma(1);
    stash_from(g0a, g0b, 0);
    __syncthreads();
  }
  mma(0);
  if (k + 1 < nk) {
    stash_from(g1a, g1b, 1);
    __syncthreads();
    mma(1);
  }
  // the cache blocks of this wave's two 64 x 64 blocks (the slots of the
  // four-wave kernels' waves 2 sub + wc), after the loop
  const int64_t tix = (int64_t)I * p.NT - (int64_t)I * (I - 1) / 2 + (J - I);
  u32x4 pk0[8], pk1[8];
  dcache_load(p.gcache, tix, pk0, wc * 64 + lane);
  dcache_load(p.gcache, tix, pk1, (2 + wc) * 64 + lane);
  wave_epilogue<0, true>(pk0, acc[0], termA, termB, I, J, p, 0.0f, 0.0f, red_v, red_i, red_j, wc);
  wave_epilogue<0, true>(pk1, acc[1], termA, termB, I, J, p, 0.0f, 0.0f, red_v, red_i, red_j, 2 + wc);
  tile_record(I, J, p, red_v, red_i, red_j);
}

// The fill of a fit's compact cache: each tile's BF16 split point Gram,
// turned into the pairs' D2lo with the point row terms and stored as
// c / D2lo rounded up to FP16 (dcache_code).  The Gram runs over all the
// points' chunks with the next two in flight, on 256 x 256 quads of four
// tiles, one workgroup of eight waves per quad: the four tiles share their
// two row panels and two column panels, so every chunk staged through LDS
// feeds twice the MFMA work of a one-tile workgroup, halving the panel
// traffic from L2 and, for wide rows (a BF16 split row of 4096 coordinates
// is 16 KB, a panel 2 MB), from HBM.  Wave w holds rows 64 (w & 1) .. + 63 of tile w >> 2 (row) / (w >> 1)
// & 1 (column) of the quad, all 128 columns, as 2 x 4 blocks: the blocks of
// two 64 x 64 waves of the one-tile kernels, stored to the same slots.  Rows
// past the last tile (odd tile counts) are read from the last row and their
// tiles, like the quad's tile below the diagonal, are not stored.  The
// launch passes the quad triangle's super-tile rows and slots in p.NS and
// p.nslots.
constexpr int QT = 2 * kTile;   // rows of a quad
__global__ __launch_bounds__(512) void k_pairs_bf16x3_fill_quad(PairsArgsB b) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  unsigned char* As = lds_raw;                          // [2][256][WROW]
  unsigned char* Bs = lds_raw + 2 * QT * WROW;          // [2][256][WROW]
  float* loA = reinterpret_cast<float*>(lds_raw + 4 * QT * WROW);   // lo of D^2 row terms, quad rows
  float* loB = loA + QT;                                            // and quad columns
  const PairsArgs p = b.p;
  const __bf16* const Xg = b.X;
  const int ldx = b.ldx, nk = b.nchx;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int dI = w >> 2, dJ = (w >> 1) & 1, h = w & 1, li = lane & 31, lh = lane >> 5;
  const int NQ = (p.NT + 1) / 2, n_pad = p.NT * kTile;

  const uint32_t G = gridDim.x;
  const int64_t slot = (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  if (slot >= p.nslots) return;
  const TilePos qp = slot_tile(slot, NQ, p.NS);
  if (qp.I < 0) return;
  const int row0 = (int)qp.I * QT, col0 = (int)qp.J * QT;

  // staging: thread t loads segment t % 4 of quad rows t / 4 and t / 4 + 128
  // of the row panels and of the column panels
  const int seg = tid & 3, lr = tid >> 2;
  const size_t xstride = (size_t)2 * ldx;
  auto row_ptr = [&](int r) { return Xg + (size_t)(r < n_pad ? r : n_pad - 1) * xstride + seg * 8; };
  const __bf16* xa0 = row_ptr(row0 + lr);
  const __bf16* xa1 = row_ptr(row0 + lr + kTile);
  const __bf16* xb0 = row_ptr(col0 + lr);
  const __bf16* xb1 = row_ptr(col0 + lr + kTile);
  auto fetch_into = [&](u32x4 (&g)[4], int c) __attribute__((always_inline)) {
    const size_t off = (size_t)c * 2 * BK;
    g[0] = *reinterpret_cast<const u32x4*>(xa0 + off);
    g[1] = *reinterpret_cast<const u32x4*>(xa1 + off);
    g[2] = *reinterpret_cast<const u32x4*>(xb0 + off);
    g[3] = *reinterpret_cast<const u32x4*>(xb1 + off);
  };
  auto stash_from = [&](const u32x4 (&g)[4], int buf) __attribute__((always_inline)) {
    unsigned char* A0 = As + (size_t)buf * QT * WROW;
    unsigned char* B0 = Bs + (size_t)buf * QT * WROW;
    *reinterpret_cast<u32x4*>(A0 + wide_at(lr, seg)) = g[0];
    *reinterpret_cast<u32x4*>(A0 + wide_at(lr + kTile, seg)) = g[1];
    *reinterpret_cast<u32x4*>(B0 + wide_at(lr, seg)) = g[2];
    *reinterpret_cast<u32x4*>(B0 + wide_at(lr + kTile, seg)) = g[3];
  };
  // acc[wc][x][y]: rows 128 dI + 64 h + 32 x, columns 128 dJ + 64 wc + 32 y
  f32x16 acc[2][2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[a][x][y] = (f32x16){0};
  // one k-step: lanes 0-31 take columns 0-7 (segment 0: hi, 2: lo), lanes
  // 32-63 columns 8-15 (segments 1 and 3)
  auto mma = [&](int buf) __attribute__((always_inline)) {
    const unsigned char* A0 = As + (size_t)buf * QT * WROW;
    const unsigned char* B0 = Bs + (size_t)buf * QT * WROW;
    bf16x8 ah[2], al[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const int r = dI * kTile + h * 64 + x * 32 + li;
      ah[x] = *reinterpret_cast<const bf16x8*>(A0 + wide_at(r, lh));
      al[x] = *reinterpret_cast<const bf16x8*>(A0 + wide_at(r, 2 + lh));
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      bf16x8 bh[2], bl[2];
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const int r = dJ * kTile + a * 64 + y * 32 + li;
        bh[y] = *reinterpret_cast<const bf16x8*>(B0 + wide_at(r, lh));
        bl[y] = *reinterpret_cast<const bf16x8*>(B0 + wide_at(r, 2 + lh));
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[a][x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[x], bh[y], acc[a][x][y], 0, 0, 0);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[a][x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[x], bl[y], acc[a][x][y], 0, 0, 0);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[a][x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[x], bh[y], acc[a][x][y], 0, 0, 0);
    }
  };

  u32x4 g0[4], g1[4];
  fetch_into(g0, 0);
  // the lo terms of the quad's 256 rows (threads 0-255) and columns (256-511)
  const int tr = tid < QT ? row0 + tid : col0 + tid - QT;
  const float lo = p.tx[tr < n_pad ? tr : n_pad - 1].x;
  if (nk > 1) fetch_into(g1, 1);
  stash_from(g0, 0);
  if (tid < QT) loA[tid] = lo;
  else loB[tid - QT] = lo;
  __syncthreads();
  int k = 0;
  for (; k + 2 < nk; k += 2) {
    fetch_into(g0, k + 2);
    mma(0);
    stash_from(g1, 1);
    __syncthreads();
    if (k + 3 < nk) fetch_into(g1, k + 3);
    mma(1);
    stash_from(g0, 0);
    __syncthreads();
  }
  mma(0);
  if (k + 1 < nk) {
    stash_from(g1, 1);
    __syncthreads();
    mma(1);
  }

  const int I = (int)qp.I * 2 + dI, J = (int)qp.J * 2 + dJ;
  if (I >= p.NT || J >= p.NT || I > J) return;   // uniform per wave
  const float c = *p.dscale;
  const int64_t tix = (int64_t)I * p.NT - (int64_t)I * (I - 1) / 2 + (J - I);
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    // D2lo = (lo_i + lo_j) - 2 g for the block of the one-tile kernels' wave
    // (h, a), then its slots
    const float b0 = loB[dJ * kTile + a * 64 + li], b1 = loB[dJ * kTile + a * 64 + 32 + li];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float av = loA[dI * kTile + h * 64 + x * 32 + (v >> 2) * 8 + lh * 4 + (v & 3)];
        acc[a][x][0][v] = fmaf(-2.0f, acc[a][x][0][v], av + b0);
        acc[a][x][1][v] = fmaf(-2.0f, acc[a][x][1][v], av + b1);
      }
    dcache_store(p.gcache, tix, acc[a], c, (h * 2 + a) * 64 + lane);
  }
}

// Constant c of a compact cache: the power of two with
// 2^-12 max_i N_i < c <= 2^-11 max_i N_i, clamped to [2^-120, 2^120] (row
// norms whose squares pass FP32's range make the FP32 row terms infinite, and
// those pairs are re-examined anyway).  Every D2lo <= D^2 <= 4 max N then
// gives c / D2lo > 2^-14, an FP16 normal, and the scalings by c and 1/c are
// exact.
__global__ __launch_bounds__(1024) void k_dcache_scale(const double* __restrict__ nx, int64_t n,
                                                       float* __restrict__ scale) {
  __shared__ double red[16];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) m = fmax(m, nx[i]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 16; ++w) m = fmax(m, red[w]);
    int e = -120;
    if (m > 0.0) {
      frexp(m * 0x1p-12, &e);   // 2^-12 m = f 2^e, f in [0.5, 1): 2^-12 m < 2^e <= 2^-11 m
      e = e < -120 ? -120 : (e > 120 ? 120 : e);
    }
    scale[0] = ldexpf(1.0f, e);
  }
}

constexpr size_t kLdsBf16 = 4 * kTile * WROW + 2 * kTile * sizeof(float4) + 3 * 8 * sizeof(float);
constexpr size_t kLdsWide = 4 * kTile * WROW + 2 * kTile * sizeof(float4) + 3 * 8 * sizeof(float);
constexpr size_t kLdsQuad = 4 * QT * WROW + 2 * QT * sizeof(float);

hipError_t launch_split_bf16(const float* src, int64_t n_pad, int64_t m, int64_t lds, int64_t ldb, __bf16* dst,
                             hipStream_t st) {
  k_split_bf16<<<(unsigned)((n_pad * ldb + 255) / 256), 256, 0, st>>>(src, n_pad, m, lds, ldb, dst);
  return hipGetLastError();
}

hipError_t launch_dcache_scale(const double* nx, int64_t n, float* scale, hipStream_t st) {
  k_dcache_scale<<<1, 1024, 0, st>>>(nx, n, scale);
  return hipGetLastError();
}

static hipError_t bf16_attrs() {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pairs_bf16x3<0>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBf16);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pairs_bf16x3_fill_quad),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsQuad);
    if (e != hipSuccess) return e;
    attr = true;
  }
  return hipSuccess;
}

hipError_t launch_pairs_screen_bf16(const PairsViewB& v, TileRec* recs, float* gcache, int gmode,
                                    const ScreenStop* stop, hipStream_t st) {
  // the compact cache is filled by launch_pairs_gram_fill_bf16 only
  if (gcache && (gmode == 1 || v.dscale == nullptr)) return hipErrorInvalidValue;
  hipError_t e0 = bf16_attrs();
  if (e0 != hipSuccess) return e0;
  const int NS = (v.NT + 7) / 8;
  const int64_t nslots = (int64_t)NS * (NS + 1) / 2 * 64;
  PairsArgsB a;
  a.X = v.Xb; a.ldx = v.ldx; a.nchx = v.ldx / BK;
  a.Y = v.Yb; a.ldy = v.ldy; a.nchy = v.ldy / BK;
  a.p = PairsArgs{nullptr, 0, 0, nullptr, 0, 0, v.tx, v.ty, v.n, v.NT, v.ntiles, NS, nslots, recs,
                  nullptr, nullptr, nullptr, 0u, nullptr, gcache, gcache ? gmode : 0,
                  nullptr, nullptr, 3.0e38f, -1.0f, v.dscale};
  if (stop) {
    a.p.stop = stop->count; a.p.stop_pairs = stop->pairs; a.p.stop_hi = stop->q_hi; a.p.stop_lo = stop->q_lo;
  }
  const int64_t G = round_up(nslots, 8);
  // the pipelined image loop needs at least one image chunk
  if (a.p.gmode == 2 && a.nchy >= 1) k_pairs_bf16x3_wide<<<(unsigned)G, 128, kLdsWide, st>>>(a);
  else k_pairs_bf16x3<0><<<(unsigned)G, 256, kLdsBf16, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_pairs_gram_fill_bf16(const PairsViewB& v, float* gcache, hipStream_t st) {
  if (!gcache || !v.dscale) return hipErrorInvalidValue;
  hipError_t e0 = bf16_attrs();
  if (e0 != hipSuccess) return e0;
  const int NS = (v.NT + 7) / 8;
  const int64_t nslots = (int64_t)NS * (NS + 1) / 2 * 64;
  PairsArgsB a;
  a.X = v.Xb; a.ldx = v.ldx; a.nchx = v.ldx / BK;
  a.Y = v.Xb; a.ldy = 0; a.nchy = 0;
  a.p = PairsArgs{nullptr, 0, 0, nullptr, 0, 0, v.tx, v.tx, v.n, v.NT, v.ntiles, NS, nslots, nullptr,
                  nullptr, nullptr, nullptr, 0u, nullptr, gcache, 1, nullptr, nullptr, 3.0e38f, -1.0f, v.dscale};
  // quads: super-tile rows and slots of the quad triangle
  const int NQ = (v.NT + 1) / 2, NSq = (NQ + 7) / 8;
  a.p.NS = NSq;
  a.p.nslots = (int64_t)NSq * (NSq + 1) / 2 * 64;
  k_pairs_bf16x3_fill_quad<<<(unsigned)round_up(a.p.nslots, 8), 512, kLdsQuad, st>>>(a);
  return hipGetLastError();
}

}  // namespace adg
