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
// of 16 (zero columns).  Upper-triangular tiles I <= J, enumerated row-major;
// workgroup b runs on XCD b mod 8, so tile = (b mod 8) * (G / 8) + b / 8 gives
// each XCD a contiguous run of tiles that share their row block in its L2.
#include "common.h"
#include "kernels.h"

namespace adg {

constexpr int PT = kTile;   // 128
constexpr int PK = kChunk;  // 16
constexpr int PLD = 20;     // LDS row stride in floats (conflict-free b128 reads)

__device__ inline void tri_tile_p(int64_t t, int64_t NT, int64_t& I, int64_t& J) {
  double b = 2.0 * (double)NT + 1.0;
  int64_t i = (int64_t)((b - sqrt(b * b - 8.0 * (double)t)) * 0.5);
  if (i < 0) i = 0;
  if (i > NT - 1) i = NT - 1;
  while (i > 0 && i * NT - i * (i - 1) / 2 > t) --i;
  while (i + 1 < NT && (i + 1) * NT - (i + 1) * i / 2 <= t) ++i;
  I = i;
  J = i + (t - (i * NT - i * (i - 1) / 2));
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

struct PairsArgs {
  const float* X; int ldx; int nchx;   // centred points, n_pad x ldx, ldx = 16 * nchx
  const float* Y; int ldy; int nchy;   // centred images, n_pad x ldy
  const float2* tx; const float2* ty;  // per-row (lo, hi) terms of D^2 and E^2
  int n; int NT; int64_t ntiles;
  TileRec* recs;                       // MODE 0
  const uint32_t* list;                // MODE 1: flagged tiles
  const CertDev* cd;                   //         thresholds and count
  int2* cand; uint32_t cap; uint32_t* ncand;
};

template <int MODE>
__global__ __launch_bounds__(256, 2) void k_pairs_f32(PairsArgs p) {
  __shared__ __attribute__((aligned(16))) float As[2][PT * PLD];
  __shared__ __attribute__((aligned(16))) float Bs[2][PT * PLD];
  __shared__ float4 termA[PT], termB[PT];
  __shared__ float red_v[2][4];
  __shared__ int red_i[2][4], red_j[2][4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 31, lh = lane >> 5;
  const int total = p.nchx + p.nchy;

  int64_t t;
  uint32_t u = blockIdx.x, u_end = 1;
  float thr_hi = 0.f, thr_lo = 0.f;
  if (MODE == 0) {
    const uint32_t G = gridDim.x;
    t = (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
    if (t >= p.ntiles) return;
  } else {
    u_end = p.cd->n_flagged;
    thr_hi = p.cd->thr_hi;
    thr_lo = p.cd->thr_lo;
    if (u >= u_end) return;
  }

  for (;;) {
    if (MODE == 1) t = p.list[u];
    int64_t I, J;
    tri_tile_p(t, p.NT, I, J);
    const int64_t row0 = I * PT, col0 = J * PT;

    if (tid < PT) {
      const float2 a = p.tx[row0 + tid], b = p.ty[row0 + tid];
      termA[tid] = make_float4(a.x, a.y, b.x, b.y);
    } else {
      const float2 a = p.tx[col0 + tid - PT], b = p.ty[col0 + tid - PT];
      termB[tid - PT] = make_float4(a.x, a.y, b.x, b.y);
    }

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
    float4 ga0, ga1, gb0, gb1;
    auto fetch = [&](int c) {
      const float* src;
      int64_t ld, cb;
      if (c < p.nchx) { src = p.X; ld = p.ldx; cb = (int64_t)c * PK; }
      else { src = p.Y; ld = p.ldy; cb = (int64_t)(c - p.nchx) * PK; }
      ga0 = *reinterpret_cast<const float4*>(src + (row0 + lr) * ld + cb + lc);
      ga1 = *reinterpret_cast<const float4*>(src + (row0 + lr + 64) * ld + cb + lc);
      gb0 = *reinterpret_cast<const float4*>(src + (col0 + lr) * ld + cb + lc);
      gb1 = *reinterpret_cast<const float4*>(src + (col0 + lr + 64) * ld + cb + lc);
    };
    auto stash = [&](int buf) {
      *reinterpret_cast<float4*>(&As[buf][lr * PLD + lc]) = ga0;
      *reinterpret_cast<float4*>(&As[buf][(lr + 64) * PLD + lc]) = ga1;
      *reinterpret_cast<float4*>(&Bs[buf][lr * PLD + lc]) = gb0;
      *reinterpret_cast<float4*>(&Bs[buf][(lr + 64) * PLD + lc]) = gb1;
    };
    // MFMA step kk sums columns kk (lanes 0-31) and 8 + kk (lanes 32-63) of
    // the chunk; the same permutation is used for both operands.
    auto mma = [&](f32x16 (&acc)[2][2], int buf) {
      float a[2][8], b[2][8];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const float* pa = &As[buf][(wr * 64 + x * 32 + li) * PLD + lh * 8];
        const float* pb = &Bs[buf][(wc * 64 + x * 32 + li) * PLD + lh * 8];
        const float4 a0 = *reinterpret_cast<const float4*>(pa), a1 = *reinterpret_cast<const float4*>(pa + 4);
        const float4 b0 = *reinterpret_cast<const float4*>(pb), b1 = *reinterpret_cast<const float4*>(pb + 4);
        a[x][0] = a0.x; a[x][1] = a0.y; a[x][2] = a0.z; a[x][3] = a0.w;
        a[x][4] = a1.x; a[x][5] = a1.y; a[x][6] = a1.z; a[x][7] = a1.w;
        b[x][0] = b0.x; b[x][1] = b0.y; b[x][2] = b0.z; b[x][3] = b0.w;
        b[x][4] = b1.x; b[x][5] = b1.y; b[x][6] = b1.z; b[x][7] = b1.w;
      }
#pragma unroll
      for (int kk = 0; kk < 8; ++kk)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[x][kk], b[y][kk], acc[x][y], 0, 0, 0);
    };

    fetch(0);
    stash(0);
    __syncthreads();
    for (int c = 0; c < total; ++c) {
      const int buf = c & 1;
      if (c + 1 < total) fetch(c + 1);
      if (c < p.nchx) mma(accX, buf);
      else mma(accY, buf);
      if (c + 1 < total) stash(buf ^ 1);
      __syncthreads();
    }

    // ------------------------------------------------------------ epilogue
    // D layout of v_mfma_f32_32x32x2f32: lane l, register v ->
    // row (v / 4) * 8 + (l / 32) * 4 + v % 4, column l % 32.
    const bool interior = (I < J) && (col0 + PT <= p.n);
    float best_hi = -1.0f, best_lo = 3.0e38f;
    int code_hi = -1, code_lo = -1;
    float4 tb[2];
    tb[0] = termB[wc * 64 + li];
    tb[1] = termB[wc * 64 + 32 + li];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rl = wr * 64 + x * 32 + (v >> 2) * 8 + lh * 4 + (v & 3);
        const float4 ta = termA[rl];
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const int cl = wc * 64 + y * 32 + li;
          const bool valid = interior || ((I < J || rl < cl) && col0 + cl < p.n);
          const float gx = accX[x][y][v], gy = accY[x][y][v];
          const float d2lo = fmaf(-2.0f, gx, ta.x + tb[y].x);
          const float d2hi = fmaf(-2.0f, gx, ta.y + tb[y].y);
          const float e2lo = fmaf(-2.0f, gy, ta.z + tb[y].z);
          const float e2hi = fmaf(-2.0f, gy, ta.w + tb[y].w);
          float qhi, qlo;
          if (d2hi <= 0.0f) { qhi = 1.0f; qlo = 1.0f; }          // identical points: skipped
          else {
            qhi = d2lo > 0.0f ? e2hi * __builtin_amdgcn_rcpf(d2lo) : 3.0e38f;
            qlo = fmaxf(e2lo, 0.0f) * __builtin_amdgcn_rcpf(d2hi);
          }
          if (MODE == 0) {
            const int code = (x * 2 + y) * 16 + v;
            if (valid && qhi > best_hi) { best_hi = qhi; code_hi = code; }
            if (valid && qlo < best_lo) { best_lo = qlo; code_lo = code; }
          } else {
            if (valid && (qhi >= thr_hi || qlo <= thr_lo)) {
              const uint32_t pos = atomicAdd(p.ncand, 1u);
              if (pos < p.cap) p.cand[pos] = make_int2((int)(row0 + rl), (int)(col0 + cl));
            }
          }
        }
      }

    if (MODE == 0) {
      auto decode = [&](int code, int& gi, int& gj) {
        if (code < 0) { gi = 0x7fffffff; gj = 0x7fffffff; return; }
        const int x = code >> 5, y = (code >> 4) & 1, v = code & 15;
        gi = (int)(row0 + wr * 64 + x * 32 + (v >> 2) * 8 + lh * 4 + (v & 3));
        gj = (int)(col0 + wc * 64 + y * 32 + li);
      };
      int ih, jh, il, jl;
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
        TileRec rec;
        rec.qhi = vh; rec.qlo = vl;
        rec.ihi = ih0 == 0x7fffffff ? -1 : ih0; rec.jhi = ih0 == 0x7fffffff ? -1 : jh0;
        rec.ilo = il0 == 0x7fffffff ? -1 : il0; rec.jlo = il0 == 0x7fffffff ? -1 : jl0;
        rec.pad0 = 0; rec.pad1 = 0;
        p.recs[t] = rec;
      }
      return;
    }
    u += gridDim.x;
    if (u >= u_end) return;
    __syncthreads();  // LDS terms / buffers are rewritten by the next tile
  }
}

hipError_t launch_pairs_screen(const PairsView& v, TileRec* recs, hipStream_t st) {
  PairsArgs a{v.X, v.ldx, v.ldx / PK, v.Y, v.ldy, v.ldy / PK, v.tx, v.ty, v.n, v.NT, v.ntiles,
              recs, nullptr, nullptr, nullptr, 0u, nullptr};
  const int64_t G = round_up(v.ntiles, 8);
  k_pairs_f32<0><<<(unsigned)G, 256, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_pairs_emit(const PairsView& v, const uint32_t* list, const CertDev* cd, int2* cand,
                             uint32_t cap, uint32_t* ncand, int grid, hipStream_t st) {
  PairsArgs a{v.X, v.ldx, v.ldx / PK, v.Y, v.ldy, v.ldy / PK, v.tx, v.ty, v.n, v.NT, v.ntiles,
              nullptr, list, cd, cand, cap, ncand};
  k_pairs_f32<1><<<(unsigned)grid, 256, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace adg
