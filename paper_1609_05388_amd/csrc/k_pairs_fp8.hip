// Step a10 (precision form, large scale): an FP8 all-pairs screen.
//
// Every centred row a_i is scaled by s_i = max_l |a_il| / 448 and quantised
// to OCP FP8 e4m3 (round to nearest even; 448 is the largest finite value):
// q_i = e4m3(a_i / s_i).  The Gram q_i . q_j runs on the unscaled
// v_mfma_f32_32x32x64_f8f6f4 (the scaled builtin with zero scale operands,
// which the compiler emits as the unscaled instruction; the same products as
// the scaled one with unit scales, about 3% faster) with FP32
// accumulation, and the epilogue forms the central estimates
//   D~^2 = N_i + N_j - 2 s_i s_j q_i.q_j,   N_i = s_i^2 |q_i|^2 (FP64, rounded),
// and the same for the images, q~ = E~^2 / D~^2.  With a 2^-4 unit roundoff
// these are estimates, not bounds: the screen ranks tiles.  Every tile keeps
// its largest and smallest q~ (the tile record); the tiles whose estimated
// distortion max(sqrt(q~hi) - 1, 1 - sqrt(q~lo)) is among the K largest are
// selected by a histogram of the keys' top 16 bits.  The certificate code then
// re-screens the selected tiles with the FP32 Gram and its rigorous bounds and
// re-evaluates in FP64 every pair there that can reach the best exact value:
// the result is the exact maximum over the selected tiles, a screened value.
//
// Operand layout in HBM: per row, chunks of 64 e4m3 bytes (one MFMA k-step);
// LDS rows hold one chunk (64 bytes, unpadded, XOR-swizzled by 16-byte
// segment: fp8_at), free of bank conflicts for the staging stores and the
// operand reads; a workgroup needs 36 KB of LDS.
#include "common.h"
#include "kernels.h"
#include "pairs_common.h"

namespace adg {

constexpr int FK = 64;               // columns per chunk (one MFMA k-step)
constexpr int FSEGS = FK / 16;       // 16-byte segments per row and chunk
constexpr int FSROWS = 256 / FSEGS;  // rows one staging pass covers
constexpr int FSPASS = kTile / FSROWS;
// LDS rows of one chunk are 64 bytes, unpadded: segment s of row r sits in
// slot s ^ ((r >> 2) & 3), so that 16 consecutive rows (16 lanes' operand
// reads) and four consecutive rows' four segments (16 lanes' staging
// stores) each cover all 64 banks.
constexpr int FROW = FK;
__device__ inline int fp8_at(int row, int seg) { return row * FROW + ((seg ^ ((row >> 2) & 3)) << 4); }

// OCP FP8 e4m3 (bias 7, no infinities, 448 the largest finite): round to
// nearest even of |x| <= 448, returned as its bit pattern.
__device__ inline unsigned char e4m3_rne(float x) {
  const unsigned s = x < 0.0f ? 0x80u : 0u;
  float a = fabsf(x);
  if (!(a > 0.0f)) return (unsigned char)s;
  if (a >= 448.0f) return (unsigned char)(s | 0x7Eu);
  int e;
  frexpf(a, &e);             // a = f * 2^e, f in [0.5, 1): unit exponent e - 1
  int ue = e - 1;
  if (ue < -6) ue = -6;      // subnormal spacing 2^-9
  const float ulp = ldexpf(1.0f, ue - 3);
  const float m = rintf(a / ulp);   // integer mantissa incl. leading bit (8..16 normal)
  float v = m * ulp;
  if (v > 448.0f) v = 448.0f;
  // encode v
  int ve;
  frexpf(v, &ve);
  int vu = ve - 1;
  unsigned bits;
  if (v == 0.0f) bits = 0u;
  else if (vu < -6) bits = (unsigned)(v / ldexpf(1.0f, -9));          // subnormal: m * 2^-9, m < 8
  else bits = ((unsigned)(vu + 7) << 3) | ((unsigned)(v / ldexpf(1.0f, vu) * 8.0f) & 7u);
  return (unsigned char)(s | bits);
}

__device__ inline float e4m3_value(unsigned char b) {
  const float sg = (b & 0x80u) ? -1.0f : 1.0f;
  const int ex = (b >> 3) & 15, mt = b & 7;
  if (ex == 0) return sg * ldexpf((float)mt, -9);
  return sg * ldexpf(1.0f + mt / 8.0f, ex - 7);
}

// One wave per row: scale, quantise into the chunked layout (ldq bytes per
// row, ldq a multiple of 128, zero padding), and the row's N = s^2 |q|^2.
__global__ void k_quant_fp8(const float* __restrict__ src, int64_t n_pad, int64_t m, int64_t lds, int64_t ldq,
                            unsigned char* __restrict__ q, float* __restrict__ scale, double* __restrict__ norm2) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n_pad) return;
  const float* a = src + row * lds;
  float mx = 0.0f;
  for (int64_t l = lane; l < m; l += 64) mx = fmaxf(mx, fabsf(a[l]));
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  const float s = mx > 0.0f ? mx / 448.0f : 1.0f;
  double acc = 0.0;
  for (int64_t l = lane; l < ldq; l += 64) {
    unsigned char b = 0;
    if (l < m) b = e4m3_rne(a[l] / s);
    q[row * ldq + l] = b;
    const double v = (double)e4m3_value(b);
    acc += v * v;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) {
    scale[row] = s;
    norm2[row] = acc * ((double)s * (double)s);   // s^2 is exact in FP64
  }
}

// Per-row epilogue terms (N_x, N_y, -2 s_x, -2 s_y); sx null: unit point
// scales (the point Gram then comes unscaled from a BF16 split cache).
__global__ void k_fp8_terms(const double* __restrict__ nx, const double* __restrict__ ny,
                            const float* __restrict__ sx, const float* __restrict__ sy, int64_t n_pad,
                            float4* __restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n_pad) t[i] = make_float4((float)nx[i], (float)ny[i], sx ? -2.0f * sx[i] : -2.0f, -2.0f * sy[i]);
}

struct PairsArgsF {
  const unsigned char* X; int ldx; int nchx;   // e4m3 points, ldx bytes per row, nchx = ldx / FK
  const unsigned char* Y; int ldy; int nchy;
  const float4* terms;                         // (N_x, N_y, -2 s_x, -2 s_y) per row
  int n; int NT; int NS; int64_t nslots;
  TileRec* recs;
  float* gcache; int gmode;                    // compact D^2 cache of the fit: 0 off, 2 load
  const float* dscale;                         // its scale (device)
};

// Epilogue of one wave's 64 x 64 block of a tile (rows 64 wr, columns 64 wc
// of tile (I, J)): the central estimates q~ of its pairs, the largest and
// smallest as sortable keys (value bits with the low 6 mantissa bits replaced
// by the pair's code), reduced over the wave into red_*[blk] (largest) and
// red_*[4 + blk] (smallest), the values scaled by sc.  Pairs whose estimated
// distance is not positive are not ranked.  LOADED: c / D2lo from the cache
// block pk, accX unused.
template <bool LOADED>
__device__ __attribute__((always_inline)) inline void fp8_block(const f32x16 (&accX)[2][2],
                                                                const f32x16 (&accY)[2][2], const u32x4 (&pk)[8],
                                                                const float4* termA, const float4* termB, int wr,
                                                                int wc, int I, int J, int n, float sc, float* red_v,
                                                                int* red_i, int* red_j, int blk) {
  const int lane = threadIdx.x & 63, li = lane & 31, lh = lane >> 5;
  const int row0 = I * kTile, col0 = J * kTile;
  const bool masked = !((I < J) && (col0 + kTile <= n));
  uint32_t khi = 0u, klo = 0xFFFFFFFFu;
  // column terms with s in place of -2 s (the row term carries the -2)
  float4 tb0 = termB[wc * 64 + li], tb1 = termB[wc * 64 + 32 + li];
  tb0.z *= -0.5f; tb0.w *= -0.5f;
  tb1.z *= -0.5f; tb1.w *= -0.5f;
  // the pass over the thread's 64 pairs, compiled once with the edge mask
  // and once without (the mask is uniform per tile: no per-pair branch)
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
          const float4 tb = y ? tb1 : tb0;
          const float e2 = fmaf(ta.w * tb.w, accY[x][y][v], ta.y + tb.y);
          // q~ = E~^2 / D~^2 with D~^2 = -2 s_i s_j g + N_i + N_j, or c q~ =
          // E~^2 g from the cached g = c / D2lo (finite: D2lo > 0)
          float q;
          bool ok;
          if constexpr (LOADED) {
            const float g = dcache_g(pk, x, y, v);
            q = e2 * g;
            ok = __float_as_uint(g) < 0x7F800000u;
          } else {
            const float d2 = fmaf(ta.z * tb.z, accX[x][y][v], ta.x + tb.x);
            q = e2 * __builtin_amdgcn_rcpf(d2);
            ok = d2 > 0.0f;
          }
          // negative estimates rank as 0 (integer max on the bits)
          const int32_t qi = __float_as_int(q);
          const uint32_t k = pair_key(__int_as_float(qi > 0 ? qi : 0), (x * 2 + y) * 16 + v);
          if (M) {
            const int cl = wc * 64 + y * 32 + li;
            ok = ok && (I < J || rl < cl) && col0 + cl < n;
          }
          khi = ok && k > khi ? k : khi;
          klo = ok && k < klo ? k : klo;
          asm volatile("" : "+v"(khi), "+v"(klo));
        }
      }
  };
  if (masked) scan(std::integral_constant<bool, true>{});
  else scan(std::integral_constant<bool, false>{});
  auto decode = [&](int code, int& gi, int& gj) {
    if (code < 0) { gi = 0x7fffffff; gj = 0x7fffffff; return; }
    const int x = code >> 5, y = (code >> 4) & 1, v = code & 15;
    gi = row0 + wr * 64 + x * 32 + (v >> 2) * 8 + lh * 4 + (v & 3);
    gj = col0 + wc * 64 + y * 32 + li;
  };
  // the wave's extreme keys and the lowest lanes holding them
  const uint32_t whi = wave_max_u32(khi), wlo = wave_min_u32(klo);
  const uint64_t bh = __ballot(khi == whi), bl = __ballot(klo == wlo);
  const int lhi = __ffsll((unsigned long long)bh) - 1, llo = __ffsll((unsigned long long)bl) - 1;
  int ih, jh, il, jl;
  decode(khi == 0u ? -1 : (int)(khi & 63u), ih, jh);
  decode(klo == 0xFFFFFFFFu ? -1 : (int)(klo & 63u), il, jl);
  ih = __shfl(ih, lhi, 64); jh = __shfl(jh, lhi, 64);
  il = __shfl(il, llo, 64); jl = __shfl(jl, llo, 64);
  if (lane == 0) {
    red_v[blk] = whi == 0u ? -1.0f : key_lo_value(whi) * sc; red_i[blk] = ih; red_j[blk] = jh;
    red_v[4 + blk] = wlo == 0xFFFFFFFFu ? 3.0e38f : key_lo_value(wlo) * sc; red_i[4 + blk] = il;
    red_j[4 + blk] = jl;
  }
}

// The tile record from its four blocks' extremes (one thread).
__device__ inline void fp8_tile_record(const float* red_v, const int* red_i, const int* red_j, TileRec* rec_out) {
  float vh = red_v[0], vl = red_v[4];
  int ih0 = red_i[0], jh0 = red_j[0], il0 = red_i[4], jl0 = red_j[4];
  for (int w = 1; w < 4; ++w) {
    if (red_v[w] > vh || (red_v[w] == vh && idx_better(red_i[w], red_j[w], ih0, jh0))) {
      vh = red_v[w]; ih0 = red_i[w]; jh0 = red_j[w];
    }
    if (red_v[4 + w] < vl || (red_v[4 + w] == vl && idx_better(red_i[4 + w], red_j[4 + w], il0, jl0))) {
      vl = red_v[4 + w]; il0 = red_i[4 + w]; jl0 = red_j[4 + w];
    }
  }
  const bool none_hi = ih0 == 0x7fffffff || vh < 0.0f;
  const bool none_lo = il0 == 0x7fffffff || vl >= 3.0e38f;
  TileRec rec;
  rec.qhi = vh; rec.qlo = vl;
  rec.ihi = none_hi ? -1 : ih0; rec.jhi = none_hi ? -1 : jh0;
  rec.ilo = none_lo ? -1 : il0; rec.jlo = none_lo ? -1 : jl0;
  rec.pad0 = 0; rec.pad1 = 0;
  *rec_out = rec;
}

// LOADED: the pairs' c / D2lo come from the fit's compact cache (filled from
// the BF16 split point Gram, a far better D^2 estimate than the FP8 Gram);
// the kernel runs the image chunks only, with the next two chunks in flight
// (two register sets of staging loads; a 64-column chunk is only 4 MFMAs per
// wave, far less than a global load's latency), loads the cached block after
// them, and runs three workgroups per CU (151 VGPRs).
template <bool LOADED>
__global__ __launch_bounds__(256, LOADED ? 3 : 2) void k_pairs_fp8(PairsArgsF b) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  unsigned char* As = lds_raw;
  unsigned char* Bs = lds_raw + 2 * kTile * FROW;
  float4* termA = reinterpret_cast<float4*>(lds_raw + 4 * kTile * FROW);
  float4* termB = termA + kTile;
  float* red_v = reinterpret_cast<float*>(termB + kTile);   // [2][4]
  int* red_i = reinterpret_cast<int*>(red_v + 8);           // [2][4]
  int* red_j = red_i + 8;                                   // [2][4]
  const unsigned char* const Xg = b.X;
  const unsigned char* const Yg = b.Y;
  const int ldx = b.ldx, ldy = b.ldy, nchx = b.nchx, nchy = b.nchy, n = b.n, NT = b.NT;
  const int total = nchx + nchy;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 31, lh = lane >> 5;

  const uint32_t G = gridDim.x;
  const int64_t slot = (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  if (slot >= b.nslots) return;
  const TilePos tp = slot_tile(slot, NT, b.NS);
  if (tp.I < 0) return;
  const int I = (int)tp.I, J = (int)tp.J;
  const int row0 = I * kTile, col0 = J * kTile;
  // the row terms load after the first chunk's loads (both in flight at
  // once); their LDS stores follow the first stash
  float4 side_t;
  auto load_side = [&]() __attribute__((always_inline)) {
    side_t = b.terms[tid < kTile ? row0 + tid : col0 + tid - kTile];
  };
  auto store_side = [&]() __attribute__((always_inline)) {
    if (tid < kTile) termA[tid] = side_t;
    else termB[tid - kTile] = side_t;
  };

  f32x16 accX[2][2], accY[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      accX[x][y] = (f32x16){0};
      accY[x][y] = (f32x16){0};
    }
  const int seg = tid % FSEGS, lr = tid / FSEGS;
  const unsigned char* xa = Xg + (size_t)(row0 + lr) * ldx + seg * 16;
  const unsigned char* xb = Xg + (size_t)(col0 + lr) * ldx + seg * 16;
  const unsigned char* ya = Yg + (size_t)(row0 + lr) * ldy + seg * 16;
  const unsigned char* yb = Yg + (size_t)(col0 + lr) * ldy + seg * 16;
  // two register sets of staging loads (the second for the pipelined image
  // loop of the LOADED kernel)
  u32x4 ga[FSPASS], gb[FSPASS], ha[FSPASS], hb[FSPASS];
  u32x4 pk[8];   // LOADED: the tile's compact cache block
  auto fetch_into = [&](u32x4 (&ra)[FSPASS], u32x4 (&rb)[FSPASS], int c) __attribute__((always_inline)) {
    if (c < nchx) {
      const size_t off = (size_t)c * FK;
#pragma unroll
      for (int m = 0; m < FSPASS; ++m) {
        ra[m] = *reinterpret_cast<const u32x4*>(xa + off + (size_t)FSROWS * m * ldx);
        rb[m] = *reinterpret_cast<const u32x4*>(xb + off + (size_t)FSROWS * m * ldx);
      }
    } else {
      const size_t off = (size_t)(c - nchx) * FK;
#pragma unroll
      for (int m = 0; m < FSPASS; ++m) {
        ra[m] = *reinterpret_cast<const u32x4*>(ya + off + (size_t)FSROWS * m * ldy);
        rb[m] = *reinterpret_cast<const u32x4*>(yb + off + (size_t)FSROWS * m * ldy);
      }
    }
  };
  auto stash_from = [&](const u32x4 (&ra)[FSPASS], const u32x4 (&rb)[FSPASS], int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int m = 0; m < FSPASS; ++m) {
      *reinterpret_cast<u32x4*>(As + (size_t)buf * kTile * FROW + fp8_at(lr + FSROWS * m, seg)) = ra[m];
      *reinterpret_cast<u32x4*>(Bs + (size_t)buf * kTile * FROW + fp8_at(lr + FSROWS * m, seg)) = rb[m];
    }
  };
  auto fetch = [&](int c) __attribute__((always_inline)) { fetch_into(ga, gb, c); };
  auto stash = [&](int buf) __attribute__((always_inline)) { stash_from(ga, gb, buf); };
  auto fetch2 = [&](int c) __attribute__((always_inline)) { fetch_into(ha, hb, c); };
  auto stash2 = [&](int buf) __attribute__((always_inline)) { stash_from(ha, hb, buf); };
  // one k-step: lanes 0-31 take bytes 0-31 of their row (segments 0, 1),
  // lanes 32-63 bytes 32-63 (segments 2, 3), the same split for both operands.
  auto mma = [&](f32x16 (&acc)[2][2], int buf) __attribute__((always_inline)) {
    const unsigned char* A0 = As + (size_t)buf * kTile * FROW;
    const unsigned char* B0 = Bs + (size_t)buf * kTile * FROW;
    {
      i32x8 av[2], bv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const int ra = wr * 64 + x * 32 + li, rb = wc * 64 + x * 32 + li;
        const u32x4 a0 = *reinterpret_cast<const u32x4*>(A0 + fp8_at(ra, 2 * lh));
        const u32x4 a1 = *reinterpret_cast<const u32x4*>(A0 + fp8_at(ra, 2 * lh + 1));
        const u32x4 b0 = *reinterpret_cast<const u32x4*>(B0 + fp8_at(rb, 2 * lh));
        const u32x4 b1 = *reinterpret_cast<const u32x4*>(B0 + fp8_at(rb, 2 * lh + 1));
        av[x] = (i32x8){(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w, (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
        bv[x] = (i32x8){(int)b0.x, (int)b0.y, (int)b0.z, (int)b0.w, (int)b1.x, (int)b1.y, (int)b1.z, (int)b1.w};
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av[x], bv[y], acc[x][y], 0, 0, 0, 0, 0, 0);
    }
  };

  const int64_t tix = (int64_t)I * NT - (int64_t)I * (I - 1) / 2 + (J - I);
  if (LOADED) {
    // image chunk k (0 <= k < nk) sits in LDS buffer k & 1 and, while in
    // flight, in register set k & 1
    const int nk = nchy;
    fetch(nchx);
    load_side();
    if (nk > 1) fetch2(nchx + 1);
    stash(0);
    store_side();
    __syncthreads();
    int k = 0;
    for (; k + 2 < nk; k += 2) {
      fetch(nchx + k + 2);
      mma(accY, 0);
      stash2(1);
      __syncthreads();
      if (k + 3 < nk) fetch2(nchx + k + 3);
      mma(accY, 1);
      stash(0);
      __syncthreads();
    }
    mma(accY, 0);
    if (k + 1 < nk) {
      stash2(1);
      __syncthreads();
      mma(accY, 1);
    }
    // the cached block after the image loop
    dcache_load(b.gcache, tix, pk, threadIdx.x);
  } else {
    fetch(0);
    load_side();
    stash(0);
    store_side();
    __syncthreads();
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

  // epilogue: central estimates, largest and smallest q~ of the tile
  const float sc = LOADED ? 1.0f / *b.dscale : 1.0f;   // exact: a power of two
  fp8_block<LOADED>(accX, accY, pk, termA, termB, wr, wc, I, J, n, sc, red_v, red_i, red_j, wave);
  __syncthreads();
  if (tid == 0) fp8_tile_record(red_v, red_i, red_j, b.recs + tix);
}

// The cached screen on 256 x 256 quads of four tiles, one workgroup of eight
// waves per quad: the four tiles share two row panels and two column panels
// of image chunks, so a chunk staged through LDS feeds twice the MFMAs of a
// one-tile workgroup, and each wave holds 64 rows x 128 columns (2 x 4
// blocks of 32 x 32) of one tile: every A fragment it reads from LDS feeds
// four MFMAs and every B fragment two (12 KB of operand reads per 8 MFMAs,
// against 8 KB per 4 with four waves of 2 x 2 blocks per tile).  Wave w
// holds rows 64 (w & 1) .. + 63 of tile (w >> 2, (w >> 1) & 1) of the quad,
// the blocks of the four-wave kernel's waves 2 (w & 1) and 2 (w & 1) + 1,
// whose cache slots it loads after the loop; the epilogue runs once per
// block and thread t < 4 writes tile t's record.  Rows past the last tile
// (odd tile counts) are read from the last row; their tiles, like the quad's
// tile below the diagonal, get no record.  The launch passes the quad
// triangle's super-tile rows and slots in b.NS and b.nslots.
constexpr int QT8 = 2 * kTile;   // rows of a quad
__global__ __launch_bounds__(512) void k_pairs_fp8_quad(PairsArgsF b) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  unsigned char* As = lds_raw;                          // [2][256][FROW]
  unsigned char* Bs = lds_raw + 2 * QT8 * FROW;         // [2][256][FROW]
  float4* termA = reinterpret_cast<float4*>(lds_raw + 4 * QT8 * FROW);   // the quad's rows
  float4* termB = termA + QT8;                                            // and columns
  float* red_v = reinterpret_cast<float*>(termB + QT8);   // [4 tiles][8]
  int* red_i = reinterpret_cast<int*>(red_v + 32);
  int* red_j = red_i + 32;
  const unsigned char* const Yg = b.Y;
  const int ldy = b.ldy, nk = b.nchy, n = b.n, NT = b.NT;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int dI = w >> 2, dJ = (w >> 1) & 1, h = w & 1, li = lane & 31, lh = lane >> 5;
  const int NQ = (NT + 1) / 2, n_pad = NT * kTile;

  const uint32_t G = gridDim.x;
  const int64_t slot = (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  if (slot >= b.nslots) return;
  const TilePos qp = slot_tile(slot, NQ, b.NS);
  if (qp.I < 0) return;
  const int row0 = (int)qp.I * QT8, col0 = (int)qp.J * QT8;

  // staging: thread t loads segment t % 4 of quad rows t / 4 and t / 4 + 128
  // of the row panel and of the column panel
  const int seg = tid & 3, lr = tid >> 2;
  auto row_ptr = [&](int r) { return Yg + (size_t)(r < n_pad ? r : n_pad - 1) * ldy + seg * 16; };
  const unsigned char* ya0 = row_ptr(row0 + lr);
  const unsigned char* ya1 = row_ptr(row0 + lr + kTile);
  const unsigned char* yb0 = row_ptr(col0 + lr);
  const unsigned char* yb1 = row_ptr(col0 + lr + kTile);
  auto fetch_into = [&](u32x4 (&g)[4], int c) __attribute__((always_inline)) {
    const size_t off = (size_t)c * FK;
    g[0] = *reinterpret_cast<const u32x4*>(ya0 + off);
    g[1] = *reinterpret_cast<const u32x4*>(ya1 + off);
    g[2] = *reinterpret_cast<const u32x4*>(yb0 + off);
    g[3] = *reinterpret_cast<const u32x4*>(yb1 + off);
  };
  auto stash_from = [&](const u32x4 (&g)[4], int buf) __attribute__((always_inline)) {
    unsigned char* A0 = As + (size_t)buf * QT8 * FROW;
    unsigned char* B0 = Bs + (size_t)buf * QT8 * FROW;
    *reinterpret_cast<u32x4*>(A0 + fp8_at(lr, seg)) = g[0];
    *reinterpret_cast<u32x4*>(A0 + fp8_at(lr + kTile, seg)) = g[1];
    *reinterpret_cast<u32x4*>(B0 + fp8_at(lr, seg)) = g[2];
    *reinterpret_cast<u32x4*>(B0 + fp8_at(lr + kTile, seg)) = g[3];
  };
  // acc[a][x][y]: rows 128 dI + 64 h + 32 x, columns 128 dJ + 64 a + 32 y
  f32x16 acc[2][2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[a][x][y] = (f32x16){0};
  // one k-step: lanes 0-31 bytes 0-31 of their row, lanes 32-63 bytes 32-63
  auto frag = [&](const unsigned char* P, int r) __attribute__((always_inline)) {
    const u32x4 q0 = *reinterpret_cast<const u32x4*>(P + fp8_at(r, 2 * lh));
    const u32x4 q1 = *reinterpret_cast<const u32x4*>(P + fp8_at(r, 2 * lh + 1));
    return (i32x8){(int)q0.x, (int)q0.y, (int)q0.z, (int)q0.w, (int)q1.x, (int)q1.y, (int)q1.z, (int)q1.w};
  };
  auto mma = [&](int buf) __attribute__((always_inline)) {
    const unsigned char* A0 = As + (size_t)buf * QT8 * FROW;
    const unsigned char* B0 = Bs + (size_t)buf * QT8 * FROW;
    i32x8 av[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) av[x] = frag(A0, dI * kTile + h * 64 + x * 32 + li);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      i32x8 bv[2];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = frag(B0, dJ * kTile + a * 64 + y * 32 + li);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[a][x][y] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av[x], bv[y], acc[a][x][y], 0, 0, 0, 0, 0, 0);
    }
  };

  u32x4 g0[4], g1[4];
  fetch_into(g0, 0);
  // the row terms of the quad's 256 rows (threads 0-255) and columns (256-511)
  const int tr = tid < QT8 ? row0 + tid : col0 + tid - QT8;
  const float4 tt = b.terms[tr < n_pad ? tr : n_pad - 1];
  if (nk > 1) fetch_into(g1, 1);
  stash_from(g0, 0);
  if (tid < QT8) termA[tid] = tt;
  else termB[tid - QT8] = tt;
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
  const float sc = 1.0f / *b.dscale;   // exact: a power of two
  const int tq = dI * 2 + dJ;
  if (I < NT && J < NT && I <= J) {   // uniform per wave
    const int64_t tix = (int64_t)I * NT - (int64_t)I * (I - 1) / 2 + (J - I);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      u32x4 pk[8];
      dcache_load(b.gcache, tix, pk, (h * 2 + a) * 64 + lane);
      fp8_block<true>(acc[a], acc[a], pk, termA + dI * kTile, termB + dJ * kTile, h, a, I, J, n, sc,
                      red_v + tq * 8, red_i + tq * 8, red_j + tq * 8, h * 2 + a);
    }
  }
  __syncthreads();
  if (tid < 4) {
    const int It = (int)qp.I * 2 + (tid >> 1), Jt = (int)qp.J * 2 + (tid & 1);
    if (It < NT && Jt < NT && It <= Jt)
      fp8_tile_record(red_v + tid * 8, red_i + tid * 8, red_j + tid * 8,
                      b.recs + ((int64_t)It * NT - (int64_t)It * (It - 1) / 2 + (Jt - It)));
  }
}

// Estimated distortion of a tile record, as a monotone 32-bit key.
__device__ inline uint32_t tile_key(const TileRec& r) {
  float u = 0.0f;
  if (r.ihi >= 0) u = fmaxf(u, sqrtf(fmaxf(r.qhi, 0.0f)) - 1.0f);
  if (r.ilo >= 0) u = fmaxf(u, 1.0f - sqrtf(fmaxf(r.qlo, 0.0f)));
  return __float_as_uint(fmaxf(u, 0.0f));   // non-negative floats order like their bits
}

// The K tiles of largest key are found on the keys' top 16 bits (bucket
// b = key >> 16) in two histogram passes of 256 buckets each: first over the
// top byte of b, then, among the tiles whose top byte is the selected one,
// over its low byte.  Each workgroup counts into LDS and adds its nonzero
// counters to the global ones.  Neighbouring tiles' keys fall in few buckets,
// so the lanes of a wave that share a bucket add their count with one LDS
// atomic: the first pending lane's bucket is broadcast, the lanes holding it
// are counted by a ballot, and they leave the loop.
// sel < 0: pass 1 (bucket b >> 8); else pass 2 (tiles with b >> 8 == *sel,
// bucket b & 255).
__global__ __launch_bounds__(256) void k_key_hist256(const TileRec* __restrict__ recs, int64_t ntiles,
                                                     const uint32_t* __restrict__ sel, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x, lane = tid & 63;
  h[tid] = 0;
  __syncthreads();
  const int s = sel ? (int)sel[0] : -1;
  for (int64_t t0 = (int64_t)blockIdx.x * 256; t0 < ntiles; t0 += (int64_t)gridDim.x * 256) {
    const int64_t t = t0 + tid;
    int bk = -1;
    if (t < ntiles) {
      const uint32_t b = tile_key(recs[t]) >> 16;
      if (s < 0) bk = (int)(b >> 8);
      else if ((int)(b >> 8) == s) bk = (int)(b & 255u);
    }
    bool pending = bk >= 0;
    for (;;) {
      const uint64_t pend = __ballot(pending);
      if (pend == 0) break;
      const int leader = __ffsll((unsigned long long)pend) - 1;
      const int lb = __shfl(bk, leader, 64);
      const uint64_t same = __ballot(pending && bk == lb);
      if (lane == leader) atomicAdd(&h[lb], (uint32_t)__popcll(same));
      if (bk == lb) pending = false;
    }
  }
  __syncthreads();
  if (h[tid]) atomicAdd(&hist[tid], h[tid]);
}

// Pass-1 selection (one workgroup of 256): the largest top byte t whose
// tiles with top byte >= t number at least K (0 if there are fewer), into
// out[0], and the count of tiles above it, into out[1].
__global__ __launch_bounds__(256) void k_key_select_top(const uint32_t* __restrict__ hist, uint32_t K,
                                                        uint32_t* __restrict__ out) {
  __shared__ uint32_t suf[257];   // suf[t] = tiles with top byte >= t
  const int t = threadIdx.x;
  suf[t] = hist[t];
  if (t == 0) suf[256] = 0;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const uint32_t v = suf[t] + (t + o < 256 ? suf[t + o] : 0u);
    __syncthreads();
    suf[t] = v;
    __syncthreads();
  }
  if (suf[t] >= K && suf[t + 1] < K) {   // exactly one such t, when any
    out[0] = (uint32_t)t;
    out[1] = suf[t + 1];
  }
  if (t == 0 && suf[0] < K) {
    out[0] = 0;
    out[1] = suf[1];
  }
}

// Pass-2 selection: within the selected top byte, the largest bucket b such
// that the tiles in buckets >= b number at least K (bucket 0, all tiles, if
// fewer); when the boundary bucket would take the count above kmax, b + 1
// (fewer than K tiles, none of that bucket).  thr[0] = b.
__global__ void k_key_select_low(const uint32_t* __restrict__ hist2, const uint32_t* __restrict__ top,
                                 uint32_t K, uint32_t kmax, uint32_t* __restrict__ thr) {
  if (threadIdx.x != 0) return;
  const uint32_t hb = top[0];
  uint64_t acc = top[1];
  int lo = 255;
  for (; lo > 0; --lo) {
    if (acc + hist2[lo] >= K) break;
    acc += hist2[lo];
  }
  uint32_t b = (hb << 8) | (uint32_t)lo;
  if (acc + hist2[lo] > kmax && b < 65535u) ++b;
  thr[0] = b;
}

// Tiles whose key bucket is >= the threshold and that hold a pair: their
// indices appended to list, counted in nsel.
__global__ void k_key_compact(const TileRec* __restrict__ recs, int64_t ntiles, const uint32_t* __restrict__ thr,
                              uint32_t* __restrict__ list, uint32_t* __restrict__ nsel) {
  const uint32_t tb = thr[0];
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < ntiles; t += (int64_t)gridDim.x * 256) {
    const TileRec r = recs[t];
    if ((tile_key(r) >> 16) < tb || (r.ihi < 0 && r.ilo < 0)) continue;
    list[atomicAdd(nsel, 1u)] = (uint32_t)t;
  }
}

constexpr size_t kLdsFp8 = 4 * kTile * FROW + 2 * kTile * sizeof(float4) + 24 * sizeof(float);
constexpr size_t kLdsFp8Quad = 4 * QT8 * FROW + 2 * QT8 * sizeof(float4) + 96 * sizeof(float);
// Cached screens with at least this many image chunks run on quads (one
// workgroup per CU, 10% faster at 32 chunks, 3% at 20); shorter ones on
// one-tile workgroups (three per CU: at 4 chunks the quads are 19% slower).
constexpr int kQuadMinChunks = 8;

hipError_t launch_quant_fp8(const float* src, int64_t n_pad, int64_t m, int64_t lds, int64_t ldq, unsigned char* q,
                            float* scale, double* norm2, hipStream_t st) {
  k_quant_fp8<<<(unsigned)((n_pad + 3) / 4), 256, 0, st>>>(src, n_pad, m, lds, ldq, q, scale, norm2);
  return hipGetLastError();
}

hipError_t launch_fp8_terms(const double* nx, const double* ny, const float* sx, const float* sy, int64_t n_pad,
                            float4* t, hipStream_t st) {
  k_fp8_terms<<<(unsigned)((n_pad + 255) / 256), 256, 0, st>>>(nx, ny, sx, sy, n_pad, t);
  return hipGetLastError();
}

hipError_t launch_pairs_screen_fp8(const unsigned char* Xq, int ldx, const unsigned char* Yq, int ldy,
                                   const float4* terms, int n, int NT, TileRec* recs, float* gcache, int gmode,
                                   const float* dscale, hipStream_t st) {
  if (!recs || (gcache && (gmode != 2 || dscale == nullptr))) return hipErrorInvalidValue;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pairs_fp8<false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsFp8);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pairs_fp8<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsFp8);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pairs_fp8_quad),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsFp8Quad);
    if (e != hipSuccess) return e;
    attr = true;
  }
  PairsArgsF a;
  a.X = Xq; a.ldx = ldx; a.nchx = ldx / FK;
  a.Y = Yq; a.ldy = ldy; a.nchy = ldy / FK;
  a.terms = terms;
  a.n = n; a.NT = NT;
  a.NS = (NT + 7) / 8;
  a.nslots = (int64_t)a.NS * (a.NS + 1) / 2 * 64;
  a.recs = recs;
  a.gcache = gcache;
  a.gmode = gcache ? gmode : 0;
  a.dscale = dscale;
  if (a.gmode == 2 && a.nchy >= 1 && a.nchy < kQuadMinChunks) {
    k_pairs_fp8<true><<<(unsigned)round_up(a.nslots, 8), 256, kLdsFp8, st>>>(a);
  } else if (a.gmode == 2 && a.nchy >= 1) {
    // quads: super-tile rows and slots of the quad triangle
    const int NQ = (NT + 1) / 2, NSq = (NQ + 7) / 8;
    a.NS = NSq;
    a.nslots = (int64_t)NSq * (NSq + 1) / 2 * 64;
    k_pairs_fp8_quad<<<(unsigned)round_up(a.nslots, 8), 512, kLdsFp8Quad, st>>>(a);
  } else {
    k_pairs_fp8<false><<<(unsigned)round_up(a.nslots, 8), 256, kLdsFp8, st>>>(a);
  }
  return hipGetLastError();
}

hipError_t launch_topk_tiles(const TileRec* recs, int64_t ntiles, uint32_t K, uint32_t kmax, uint32_t* hist,
                             uint32_t* thr, uint32_t* list, uint32_t* nsel, hipStream_t st) {
  int64_t g = (ntiles + 255) / 256;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  // hist: [0, 256) pass-1 counters, [256, 512) pass-2 counters, [512, 514)
  // the pass-1 selection
  hipError_t e = hipMemsetAsync(hist, 0, 512 * sizeof(uint32_t), st);
  if (e != hipSuccess) return e;
  k_key_hist256<<<(unsigned)g, 256, 0, st>>>(recs, ntiles, nullptr, hist);
  k_key_select_top<<<1, 256, 0, st>>>(hist, K, hist + 512);
  k_key_hist256<<<(unsigned)g, 256, 0, st>>>(recs, ntiles, hist + 512, hist + 256);
  k_key_select_low<<<1, 64, 0, st>>>(hist + 256, hist + 512, K, kmax, thr);
  k_key_compact<<<(unsigned)g, 256, 0, st>>>(recs, ntiles, thr, list, nsel);
  return hipGetLastError();
}

int fp8_chunk() { return FK; }

}  // namespace adg
