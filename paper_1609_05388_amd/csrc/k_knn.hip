// Exact k-nearest-neighbour queries, the operation behind the
// applications of Secs. 4.6 and 4.7: the 10-NN query of every descriptor of a query photo in the
// image-retrieval experiment and the 30-NN graph of the classification
// experiment.  For every query q the answer is the k database rows x with the
// smallest FP64 squared distance ||q - x||^2, summed coordinate by
// coordinate, equal distances ordered by the smaller database index.
//
// Stage 1, k_knn_screen: tiles of 128 database rows x 64 queries on
//   v_mfma_f32_32x32x2f32 give est = N_q + N_x - 2 q.x (FP32 norms of the FP64
//   squared norms).  A workgroup scans one split of the database for one block
//   of 64 queries and keeps, per query, the KP = 32 smallest estimates as
//   64-bit keys (order-preserving bits of est, then the database index); two
//   workgroups share a CU, so one's MFMAs overlap the other's selection.
//   Candidates below the query's current 32nd key go to an LDS queue of 64
//   slots: each lane reserves its slots for the whole tile with one atomic
//   per query, and the queues are merged into the sorted lists when one
//   passes 32 entries.  A tile whose candidates would not fit (the first
//   tiles of a scan) is taken in four sub-steps of at most 32 candidates per
//   query with a merge check after each.
// Stage 2, k_knn_finish (one wave per query): the KP smallest keys over all
//   splits, their exact FP64 distances, the k best by (distance, index), and a
//   check that no row outside the KP can enter the answer:
//     |est - d| <= c_K (N_q + N_x) <= c_K (N_q + max_x N_x) =: beta
//   for every estimate (FP32 rounding of the norms, gamma_K of the MFMA dot
//   product, the add and the fma), so every row not kept has
//   d >= est_KP - beta; the FP64 sums themselves are within (m + 4) u64 of d.
//   A query whose k-th distance is not strictly below that bound is listed.
// Stage 3, k_knn_fallback: listed queries by FP64 brute force over the whole
//   database (same distance arithmetic, same order), one workgroup each.
//
// Layout: queries and database rows are copied to row-padded FP32 panels of
// width K = m rounded up to 16 (zero columns and rows); keys of the screen are
// [query][split][KP].  Workgroup b runs on XCD b mod 8; slot =
// (b mod 8) * (G / 8) + b / 8 and slot = split * QB + query block, so the
// workgroups resident on one XCD scan the same database split and share its
// tiles in that XCD's L2.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace adg {

constexpr int KN_T = 128;     // database rows per tile
constexpr int KN_Q = kKnnQueries;  // queries per block
constexpr int KN_C = 16;      // chunk width
constexpr int KN_LD = 16;     // LDS operand row stride (floats, unpadded; see kn_at)
constexpr int KN_QC = 64;     // queue capacity per query
constexpr int KN_LST = kKnnKeep + 1;  // padded list row (u64)
constexpr uint64_t kKnnEmpty = (0xFF800000ull << 32) | 0xFFFFFFFFull;  // key of (+inf, no row)

// LDS position of float4 number q (0..3) of row `row` in a chunk buffer: the
// float4s of a row are XOR-swizzled with bits 2-3 of the row, so that the
// staging writes (4 rows x 4 float4s per 16 lanes) and the MFMA operand reads
// (16 rows x 1 float4 per 16 lanes) both hit 16 distinct 4-bank groups.
__device__ inline int kn_at(int row, int q) { return row * KN_LD + ((q ^ (row >> 2)) & 3) * 4; }

// 76,048 bytes: two workgroups share a CU's 160 KB.
struct KnnLds {
  float As[2][KN_T * KN_LD];  // database chunk
  float Bs[2][KN_Q * KN_LD];  // query chunk
  float nd[KN_T];
  float nq[KN_Q], tau[KN_Q];
  int cnt[KN_Q];
  int res[2][KN_Q];           // slots reserved by the current / previous tile
  int flag, flag2, pad0, pad1;
  uint64_t L[KN_Q * KN_LST];
  uint64_t Qu[KN_Q * KN_QC];
};

__device__ inline uint64_t knn_key(float e, uint32_t row) {
  uint32_t b = __float_as_uint(e);
  b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return ((uint64_t)b << 32) | row;
}
__device__ inline float knn_key_est(uint64_t k) {
  uint32_t b = (uint32_t)(k >> 32);
  b = (b & 0x80000000u) ? (b & 0x7fffffffu) : ~b;
  return __uint_as_float(b);
}

// Padded FP32 copy of rows [0, n) (zero rows up to n_pad), FP64 and FP32
// squared norms; one wave per row.
__global__ __launch_bounds__(256) void k_knn_prep(const float* __restrict__ src, int64_t n, int64_t m,
                                                  int64_t n_pad, int64_t K, float* __restrict__ dst,
                                                  double* __restrict__ n64, float* __restrict__ n32,
                                                  int* __restrict__ nonfinite) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n_pad) return;
  double s = 0.0;
  for (int64_t l = lane; l < K; l += 64) {
    const float v = (row < n && l < m) ? src[row * m + l] : 0.0f;
    dst[row * K + l] = v;
    s += (double)v * (double)v;
  }
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) {
    n64[row] = s;
    n32[row] = (float)s;
    if (!isfinite(s)) atomicOr(nonfinite, 1);
  }
}

// Largest FP64 norm, one workgroup.
__global__ __launch_bounds__(1024) void k_knn_max(const double* __restrict__ v, int64_t n, double* __restrict__ out) {
  __shared__ double part[16];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) m = fmax(m, v[i]);
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 16; ++w) m = fmax(m, part[w]);
    *out = fmax(m, part[0]);
  }
}

struct KnnScreenArgs {
  const float* D; const float* Q; int K; int nch;
  const float* nd32; const float* nq32;
  int64_t nd; int QB; int S; int tps; int NTd; int excl;
  uint64_t* keys;   // [nq_pad][S][KP]
  unsigned* tau_g;  // [nq_pad] order-preserving bits of the shared threshold
};

__device__ inline unsigned knn_ord(float e) {
  const unsigned b = __float_as_uint(e);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline float knn_unord(unsigned b) {
  return __uint_as_float((b & 0x80000000u) ? (b & 0x7fffffffu) : ~b);
}

// Insert the queued keys of query q into its sorted list; returns the
// list's last (32nd) key.
__device__ inline uint64_t knn_merge_one(KnnLds& sm, int q) {
  const int c = sm.cnt[q];
  sm.cnt[q] = 0;
  uint64_t* Lq = &sm.L[q * KN_LST];
  const uint64_t* Qq = &sm.Qu[q * KN_QC];
  uint64_t last = Lq[kKnnKeep - 1];
  for (int i = 0; i < c; ++i) {
    const uint64_t kv = Qq[i];
    if (kv >= last) continue;
    int pp = 0;
#pragma unroll
    for (int step = kKnnKeep / 2; step > 0; step >>= 1)
      if (Lq[pp + step - 1] < kv) pp += step;
    for (int j = kKnnKeep - 1; j > pp; --j) Lq[j] = Lq[j - 1];
    Lq[pp] = kv;
    last = Lq[kKnnKeep - 1];
  }
  return last;
}

// One workgroup: one block of 64 queries against one split of the database,
// tiles of 128 rows x 64 queries; wave w computes rows 32w .. 32w + 31 of the
// tile against all 64 queries (two 32 x 32 MFMA blocks).
__global__ __launch_bounds__(256, 2) void k_knn_screen(KnnScreenArgs p) {
  extern __shared__ __attribute__((aligned(16))) unsigned char knn_lds_raw[];
  KnnLds& sm = *reinterpret_cast<KnnLds*>(knn_lds_raw);

  const uint32_t G = gridDim.x;
  const int64_t slot = (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  if (slot >= (int64_t)p.QB * p.S) return;
  const int s = (int)(slot / p.QB), qb = (int)(slot % p.QB);
  const int t0 = s * p.tps, t1 = min(p.NTd, t0 + p.tps);
  const int q0 = qb * KN_Q;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, lh = lane >> 5;

  if (tid < KN_Q) {
    sm.nq[tid] = p.nq32[q0 + tid];
    sm.tau[tid] = __uint_as_float(0x7f800000u);
    sm.cnt[tid] = 0;
    sm.res[0][tid] = 0;
    sm.res[1][tid] = 0;
  }
  if (tid == 0) { sm.flag = 0; sm.flag2 = 0; }
  for (int e = tid; e < KN_Q * KN_LST; e += 256) sm.L[e] = kKnnEmpty;

  // loads: database rows lr and lr + 64, query row lr (threads < 256 cover
  // 64 rows x 16 columns as float4)
  const int lr = tid >> 2, lc = (tid & 3) * 4;
  const float* qa = p.Q + (size_t)(q0 + lr) * p.K + lc;
  const size_t d64 = (size_t)64 * p.K;
  float4 ga0, ga1, gb0;
  // chunk g of the scan: tile t0 + g / nch, columns (g mod nch) * 16
  auto fetch = [&](int g) __attribute__((always_inline)) {
    const int t = t0 + g / p.nch, cb = (g % p.nch) * KN_C;
    const float* da = p.D + (size_t)(t * KN_T + lr) * p.K + lc + cb;
    ga0 = *reinterpret_cast<const float4*>(da);
    ga1 = *reinterpret_cast<const float4*>(da + d64);
    gb0 = *reinterpret_cast<const float4*>(qa + cb);
  };
  auto stash = [&](int buf) __attribute__((always_inline)) {
    *reinterpret_cast<float4*>(&sm.As[buf][kn_at(lr, lc >> 2)]) = ga0;
    *reinterpret_cast<float4*>(&sm.As[buf][kn_at(lr + 64, lc >> 2)]) = ga1;
    *reinterpret_cast<float4*>(&sm.Bs[buf][kn_at(lr, lc >> 2)]) = gb0;
  };

  const int gend = (t1 - t0) * p.nch;
  fetch(0);
  stash(0);
  // the lane's two query columns
  const int qc0 = li, qc1 = 32 + li;
  __syncthreads();
  const float nq0 = sm.nq[qc0], nq1 = sm.nq[qc1];
  float tau0, tau1;

  // Row norms of the next tile and the shared threshold are loaded with the
  // next tile's first chunk and written to LDS after this tile's epilogue.
  // Any split's 32nd smallest estimate bounds the query's global 32nd
  // smallest from above, so the smallest one published so far is a valid
  // filter here too (a stale value is merely a looser one).
  float nd_next = 0.0f;
  unsigned tg_next = 0xFF800000u;
  if (tid < KN_T) sm.nd[tid] = p.nd32[t0 * KN_T + tid];
  if (tid < KN_Q) {
    tg_next = __hip_atomic_load(&p.tau_g[q0 + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sm.tau[tid] = fminf(sm.tau[tid], knn_unord(tg_next));
  }
  __syncthreads();

  for (int t = t0; t < t1; ++t) {
    const int row0 = t * KN_T;
    // the previous tile's reserved slots become committed queue entries
    // (its writes are complete: a barrier separates them from here)
    if (t > t0 && tid < KN_Q) {
      sm.cnt[tid] += sm.res[(t - 1) & 1][tid];
      sm.res[(t - 1) & 1][tid] = 0;
    }
    f32x16 acc[2];
    acc[0] = (f32x16){0};
    acc[1] = (f32x16){0};
    const int gb = (t - t0) * p.nch;
    for (int c = 0; c < p.nch; ++c) {
      const int g = gb + c, buf = g & 1;
      if (g + 1 < gend) {
        fetch(g + 1);
        if (c + 1 == p.nch) {
          if (tid < KN_T) nd_next = p.nd32[row0 + KN_T + tid];
          if (tid < KN_Q)
            tg_next = __hip_atomic_load(&p.tau_g[q0 + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      // MFMA step kk sums chunk columns kk (lanes 0-31) and 8 + kk (lanes
      // 32-63), the same permutation for both operands.
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const float4 a4 = *reinterpret_cast<const float4*>(&sm.As[buf][kn_at(wave * 32 + li, lh * 2 + half)]);
        float4 b4[2];
#pragma unroll
        for (int y = 0; y < 2; ++y)
          b4[y] = *reinterpret_cast<const float4*>(&sm.Bs[buf][kn_at(y * 32 + li, lh * 2 + half)]);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            acc[y] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[kk], b4[y][kk], acc[y], 0, 0, 0);
      }
      // the next tile's first chunk is stashed after this tile's epilogue,
      // so its loads complete behind the epilogue
      if (g + 1 < gend && c + 1 < p.nch) stash(buf ^ 1);
      __syncthreads();
    }
    tau0 = sm.tau[qc0];
    tau1 = sm.tau[qc1];

    // Edge tiles: rows past the database end, and with exclude-self the tile
    // that holds this block's queries as rows.
    const bool masked = (row0 + KN_T > p.nd) || (p.excl && q0 >= row0 && q0 < row0 + KN_T);
    // D layout: lane l, register v -> row (v / 4) * 8 + (l / 32) * 4 + v % 4,
    // column l % 32: 16 candidates per lane and query, 128 per query over the
    // 4 waves.  All 32 estimates of the lane first (straight-line code).
    float est[16][2];
    auto eval = [&](auto maskc) __attribute__((always_inline)) {
      constexpr bool M = decltype(maskc)::value;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rl = wave * 32 + (v >> 2) * 8 + lh * 4 + (v & 3);
        const float ndr = sm.nd[rl];
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          float e = fmaf(-2.0f, acc[y][v], (y ? nq1 : nq0) + ndr);
          if (M) {
            const int64_t rg = row0 + rl;
            const int qg = q0 + (y ? qc1 : qc0);
            if (rg >= p.nd || (p.excl && rg == qg)) e = __uint_as_float(0x7f800000u);
          }
          est[v][y] = e;
        }
      }
    };
    if (masked) eval(std::integral_constant<bool, true>{});
    else eval(std::integral_constant<bool, false>{});
    auto row_of = [&](int v) { return (uint32_t)(row0 + wave * 32 + (v >> 2) * 8 + lh * 4 + (v & 3)); };

    // One reservation per lane and query for the whole tile.  A tile fits
    // when every query's committed entries plus its reservations stay within
    // the queue; stamps increase, so every thread reads the flags alike (a
    // thread can only move on to set later stamps after a barrier that the
    // others reach after reading them).
    const int stampT = (t - t0) * 8 + 1;
    const int rb = t & 1;
    int n0 = 0, n1 = 0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      n0 += est[v][0] < tau0 ? 1 : 0;
      n1 += est[v][1] < tau1 ? 1 : 0;
    }
    int b0 = 0, b1 = 0;
    const int c0 = sm.cnt[qc0], c1 = sm.cnt[qc1];
    if (n0) b0 = atomicAdd(&sm.res[rb][qc0], n0);
    if (n1) b1 = atomicAdd(&sm.res[rb][qc1], n1);
    const int e0 = c0 + b0 + n0, e1 = c1 + b1 + n1;
    if ((n0 && e0 > KN_QC) || (n1 && e1 > KN_QC)) sm.flag = stampT;
    else if ((n0 && e0 > KN_QC - 32) || (n1 && e1 > KN_QC - 32)) sm.flag2 = stampT;
    __syncthreads();
    if (sm.flag != stampT) {
      // fits: write the reserved entries
      if (n0 | n1) {
        int i0 = c0 + b0, i1 = c1 + b1;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          if (est[v][0] < tau0) sm.Qu[qc0 * KN_QC + i0++] = knn_key(est[v][0], row_of(v));
          if (est[v][1] < tau1) sm.Qu[qc1 * KN_QC + i1++] = knn_key(est[v][1], row_of(v));
        }
      }
      if (sm.flag2 == stampT) {
        // more than half full somewhere: merge every queue
        __syncthreads();
        if (tid < KN_Q) {
          sm.cnt[tid] += sm.res[rb][tid];
          sm.res[rb][tid] = 0;
          const uint64_t last = knn_merge_one(sm, tid);
          const unsigned lb = (unsigned)(last >> 32);
          const unsigned old = atomicMin(&p.tau_g[q0 + tid], lb);
          sm.tau[tid] = knn_unord(min(old, lb));
        }
        __syncthreads();
        tau0 = sm.tau[qc0];
        tau1 = sm.tau[qc1];
      }
    } else {
      // Some query would overflow: drop the reservations, merge the
      // committed entries, then take the tile in four sub-steps of at most 32
      // candidates per query, each followed by a merge check.
      if (tid < KN_Q) {
        sm.res[rb][tid] = 0;
        const uint64_t last = knn_merge_one(sm, tid);
        const unsigned lb = (unsigned)(last >> 32);
        const unsigned old = atomicMin(&p.tau_g[q0 + tid], lb);
        sm.tau[tid] = knn_unord(min(old, lb));
      }
      __syncthreads();
      tau0 = sm.tau[qc0];
      tau1 = sm.tau[qc1];
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int stamp = stampT + 1 + st;
        bool any = false;
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) any |= est[st * 4 + vv][0] < tau0 || est[st * 4 + vv][1] < tau1;
        if (__builtin_amdgcn_ballot_w64(any)) {
          int m0 = 0, m1 = 0;
#pragma unroll
          for (int vv = 0; vv < 4; ++vv) {
            m0 += est[st * 4 + vv][0] < tau0 ? 1 : 0;
            m1 += est[st * 4 + vv][1] < tau1 ? 1 : 0;
          }
          int i0 = m0 ? atomicAdd(&sm.cnt[qc0], m0) : 0;
          int i1 = m1 ? atomicAdd(&sm.cnt[qc1], m1) : 0;
          if (i0 + m0 > KN_QC - 32 || i1 + m1 > KN_QC - 32) sm.flag = stamp;
#pragma unroll
          for (int vv = 0; vv < 4; ++vv) {
            const int v = st * 4 + vv;
            if (est[v][0] < tau0) sm.Qu[qc0 * KN_QC + i0++] = knn_key(est[v][0], row_of(v));
            if (est[v][1] < tau1) sm.Qu[qc1 * KN_QC + i1++] = knn_key(est[v][1], row_of(v));
          }
        }
        __syncthreads();
        if (sm.flag == stamp) {
          if (tid < KN_Q) {
            const uint64_t last = knn_merge_one(sm, tid);
            const unsigned lb = (unsigned)(last >> 32);
            const unsigned old = atomicMin(&p.tau_g[q0 + tid], lb);
            sm.tau[tid] = knn_unord(min(old, lb));
          }
          __syncthreads();
          tau0 = sm.tau[qc0];
          tau1 = sm.tau[qc1];
        }
      }
    }
    const int gn = (t + 1 - t0) * p.nch;
    if (gn < gend) {
      stash(gn & 1);
      if (tid < KN_T) sm.nd[tid] = nd_next;
      if (tid < KN_Q) sm.tau[tid] = fminf(sm.tau[tid], knn_unord(tg_next));
      __syncthreads();
    }
  }

  // Queued entries that never triggered a merge (the last tile's writes
  // complete at the barrier).
  __syncthreads();
  if (tid < KN_Q) {
    sm.cnt[tid] += sm.res[(t1 - 1) & 1][tid];
    sm.res[(t1 - 1) & 1][tid] = 0;
    const uint64_t last = knn_merge_one(sm, tid);
    atomicMin(&p.tau_g[q0 + tid], (unsigned)(last >> 32));
  }
  __syncthreads();
  for (int e = tid; e < KN_Q * kKnnKeep; e += 256) {
    const int q = e / kKnnKeep, i = e % kKnnKeep;
    p.keys[((size_t)(q0 + q) * p.S + s) * kKnnKeep + i] = sm.L[q * KN_LST + i];
  }
}

// FP64 squared distance of two FP32 rows, difference, square and sum in
// coordinate order, one rounding each (no contraction).
__device__ inline double knn_dist64(const float* __restrict__ a, const float* __restrict__ b, int64_t m) {
#pragma clang fp contract(off)
  double s = 0.0;
  for (int64_t l = 0; l < m; ++l) {
    const double df = (double)a[l] - (double)b[l];
    const double sq = df * df;
    s = s + sq;
  }
  return s;
}

__device__ inline bool knn_less(double da, int ia, double db, int ib) {
  return da < db || (da == db && ia < ib);
}

struct KnnFinishArgs {
  const uint64_t* keys; int S;
  const float* Q; const float* D; int64_t m;
  int64_t nq; int k;
  const double* nq64; const double* ndmax;
  const unsigned* tau_g;  // shared thresholds of the screen
  double cK;     // screen bound constant c_K
  double g64;    // relative bound of the FP64 sums
  int32_t* idx; double* dist;
  int* nfb; int* fb;
};

__global__ __launch_bounds__(256) void k_knn_finish(KnnFinishArgs p) {
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= p.nq) return;
  // the KP smallest of the S * KP keys: lane-local pools, KP wave minima
  constexpr int PER = kKnnMaxSplits * kKnnKeep / 64;
  uint64_t kv[PER];
  const int tot = p.S * kKnnKeep;
  const uint64_t* src = p.keys + (size_t)q * tot;
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int e = lane + 64 * t;
    kv[t] = e < tot ? src[e] : ~0ull;
  }
  uint64_t mine = ~0ull;
  for (int r = 0; r < kKnnKeep; ++r) {
    uint64_t lm = kv[0];
#pragma unroll
    for (int t = 1; t < PER; ++t) lm = kv[t] < lm ? kv[t] : lm;
    uint64_t wm = lm;
    for (int o = 32; o >= 1; o >>= 1) {
      const uint64_t w2 = __shfl_xor(wm, o, 64);
      wm = w2 < wm ? w2 : wm;
    }
    if (lane == r) mine = wm;
    if (lm == wm) {
      // remove one copy (real keys are unique; empty keys may repeat)
      bool done = false;
#pragma unroll
      for (int t = 0; t < PER; ++t)
        if (!done && kv[t] == wm) { kv[t] = ~0ull; done = true; }
    }
  }
  const uint64_t klast = __shfl(mine, kKnnKeep - 1, 64);
  const bool valid = lane < kKnnKeep && mine != ~0ull && (uint32_t)mine != 0xFFFFFFFFu;
  const int row = valid ? (int)(uint32_t)mine : 0x7fffffff;
  const double d = valid ? knn_dist64(p.Q + q * p.m, p.D + (int64_t)row * p.m, p.m) : __longlong_as_double(0x7ff0000000000000ll);
  int rank = 0;
  for (int j = 0; j < kKnnKeep; ++j) {
    const double dj = __shfl(d, j, 64);
    const int ij = __shfl(row, j, 64);
    rank += knn_less(dj, ij, d, row) ? 1 : 0;
  }
  if (lane < kKnnKeep && rank < p.k) {
    p.idx[q * p.k + rank] = row;
    p.dist[q * p.k + rank] = d;
  }
  // k-th distance: the largest of the k smallest
  double dk = (lane < kKnnKeep && rank < p.k) ? d : -1.0;
  for (int o = 32; o >= 1; o >>= 1) dk = fmax(dk, __shfl_xor(dk, o, 64));
  if (lane == 0) {
    // Every row outside the kept keys has an estimate of at least the 32nd
    // kept one or the shared threshold (rows filtered or evicted in a split).
    const bool full = (uint32_t)klast != 0xFFFFFFFFu && klast != ~0ull;
    const float e_last = fminf(full ? knn_key_est(klast) : __uint_as_float(0x7f800000u), knn_unord(p.tau_g[q]));
    bool ok = true;
    if (e_last < __uint_as_float(0x7f800000u)) {
      const double beta = p.cK * (p.nq64[q] + *p.ndmax);
      const double lower = ((double)e_last - beta) * (1.0 - p.g64);
      ok = lower > dk;
    }
    if (!ok) {
      const int at = atomicAdd(p.nfb, 1);
      p.fb[at] = (int)q;
    }
  }
}

// FP64 brute force for listed queries: each thread keeps the k best of its
// rows (sorted by (distance, index)) in LDS, then k rounds of a block-wide
// minimum over the threads' list heads.
struct KnnFallbackArgs {
  const float* Q; const float* D; int64_t m; int64_t nd; int k; int excl;
  const int* fb; int32_t* idx; double* dist;
};

__global__ __launch_bounds__(256) void k_knn_fallback(KnnFallbackArgs p) {
  __shared__ double ld[kKnnKeep][256];
  __shared__ int li[kKnnKeep][256];
  __shared__ double rv[4];
  __shared__ int ri[4], rt[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t q = p.fb[blockIdx.x];
  const float* qrow = p.Q + q * p.m;
  int cnt = 0;
  double worst = __longlong_as_double(0x7ff0000000000000ll);
  for (int64_t j = tid; j < p.nd; j += 256) {
    if (p.excl && j == q) continue;
    const double d = knn_dist64(qrow, p.D + j * p.m, p.m);
    if (cnt == p.k && !(d < worst)) continue;   // later rows lose ties
    int pos = cnt < p.k ? cnt : p.k - 1;
    while (pos > 0 && d < ld[pos - 1][tid]) {
      ld[pos][tid] = ld[pos - 1][tid];
      li[pos][tid] = li[pos - 1][tid];
      --pos;
    }
    ld[pos][tid] = d;
    li[pos][tid] = (int)j;
    if (cnt < p.k) ++cnt;
    worst = cnt == p.k ? ld[p.k - 1][tid] : worst;
  }
  int head = 0;
  for (int r = 0; r < p.k; ++r) {
    double v = head < cnt ? ld[head][tid] : __longlong_as_double(0x7ff0000000000000ll);
    int vi = head < cnt ? li[head][tid] : 0x7fffffff;
    int vt = tid;
    for (int o = 32; o >= 1; o >>= 1) {
      const double v2 = __shfl_xor(v, o, 64);
      const int i2 = __shfl_xor(vi, o, 64), t2 = __shfl_xor(vt, o, 64);
      if (knn_less(v2, i2, v, vi)) { v = v2; vi = i2; vt = t2; }
    }
    if (lane == 0) { rv[wave] = v; ri[wave] = vi; rt[wave] = vt; }
    __syncthreads();
    double bv = rv[0];
    int bi = ri[0], bt = rt[0];
    for (int w = 1; w < 4; ++w)
      if (knn_less(rv[w], ri[w], bv, bi)) { bv = rv[w]; bi = ri[w]; bt = rt[w]; }
    if (tid == bt) ++head;
    if (tid == 0) {
      p.idx[q * p.k + r] = bi;
      p.dist[q * p.k + r] = bv;
    }
    __syncthreads();
  }
}

// Majority vote per group of consecutive queries (one workgroup per group):
// each neighbour adds a vote to its database label; the answer is the label
// with most votes, the smallest label among ties.  Indices or labels out of
// range set *bad and are not counted.
__global__ __launch_bounds__(256) void k_knn_vote(const int32_t* __restrict__ nn, int64_t nq, int k,
                                                  const int32_t* __restrict__ label, int64_t nd, int n_labels,
                                                  int group, int32_t* __restrict__ out, int* __restrict__ bad) {
  extern __shared__ int hist[];
  __shared__ int bc[4], bl[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < n_labels; i += 256) hist[i] = 0;
  __syncthreads();
  const int64_t a = (int64_t)blockIdx.x * group, b = min(nq, a + group);
  for (int64_t e = a * k + tid; e < b * k; e += 256) {
    const int32_t j = nn[e];
    if (j < 0 || j >= nd) { atomicOr(bad, 1); continue; }
    const int32_t lab = label[j];
    if (lab < 0 || lab >= n_labels) { atomicOr(bad, 1); continue; }
    atomicAdd(&hist[lab], 1);
  }
  __syncthreads();
  int c = -1, l = 0x7fffffff;
  for (int i = tid; i < n_labels; i += 256)
    if (hist[i] > c) { c = hist[i]; l = i; }   // i increases: first maximum kept
  for (int o = 32; o >= 1; o >>= 1) {
    const int c2 = __shfl_xor(c, o, 64), l2 = __shfl_xor(l, o, 64);
    if (c2 > c || (c2 == c && l2 < l)) { c = c2; l = l2; }
  }
  if (lane == 0) { bc[wave] = c; bl[wave] = l; }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < 4; ++w)
      if (bc[w] > c || (bc[w] == c && bl[w] < l)) { c = bc[w]; l = bl[w]; }
    out[blockIdx.x] = l;
  }
}

// ------------------------------------------------------------ launchers
hipError_t launch_knn_prep(const float* src, int64_t n, int64_t m, int64_t n_pad, int64_t K, float* dst,
                           double* n64, float* n32, int* nonfinite, hipStream_t st) {
  k_knn_prep<<<(unsigned)((n_pad + 3) / 4), 256, 0, st>>>(src, n, m, n_pad, K, dst, n64, n32, nonfinite);
  return hipGetLastError();
}

hipError_t launch_knn_max(const double* v, int64_t n, double* out, hipStream_t st) {
  k_knn_max<<<1, 1024, 0, st>>>(v, n, out);
  return hipGetLastError();
}

hipError_t launch_knn_screen(const KnnView& v, uint64_t* keys, unsigned* tau_g, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_knn_screen),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(KnnLds));
    if (e != hipSuccess) return e;
    attr = true;
  }
  KnnScreenArgs a;
  a.D = v.Dp; a.Q = v.Qp; a.K = (int)v.K; a.nch = (int)(v.K / KN_C);
  a.nd32 = v.nd32; a.nq32 = v.nq32;
  a.nd = v.nd; a.QB = v.QB; a.S = v.S; a.tps = v.tps; a.NTd = v.NTd; a.excl = v.excl;
  a.keys = keys;
  a.tau_g = tau_g;
  const int64_t G = round_up((int64_t)v.QB * v.S, 8);
  k_knn_screen<<<(unsigned)G, 256, sizeof(KnnLds), st>>>(a);
  return hipGetLastError();
}

hipError_t launch_knn_finish(const KnnView& v, const uint64_t* keys, const float* Q, const float* D,
                             const double* nq64, const double* ndmax, const unsigned* tau_g, double cK, double g64,
                             int k, int32_t* idx, double* dist, int* nfb, int* fb, hipStream_t st) {
  KnnFinishArgs a;
  a.keys = keys; a.S = v.S; a.Q = Q; a.D = D; a.m = v.m; a.nq = v.nq; a.k = k;
  a.nq64 = nq64; a.ndmax = ndmax; a.tau_g = tau_g; a.cK = cK; a.g64 = g64;
  a.idx = idx; a.dist = dist; a.nfb = nfb; a.fb = fb;
  k_knn_finish<<<(unsigned)((v.nq + 3) / 4), 256, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_knn_fallback(const float* Q, const float* D, int64_t m, int64_t nd, int k, int excl, const int* fb,
                               int nfb, int32_t* idx, double* dist, hipStream_t st) {
  KnnFallbackArgs a{Q, D, m, nd, k, excl, fb, idx, dist};
  k_knn_fallback<<<(unsigned)nfb, 256, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_knn_vote(const int32_t* nn, int64_t nq, int k, const int32_t* label, int64_t nd, int n_labels,
                           int group, int32_t* out, int* bad, hipStream_t st) {
  const int64_t groups = (nq + group - 1) / group;
  k_knn_vote<<<(unsigned)groups, 256, (size_t)n_labels * sizeof(int), st>>>(nn, nq, k, label, nd, n_labels, group,
                                                                              out, bad);
  return hipGetLastError();
}

}  // namespace adg
