// FP64 MFMA products of the path:
//   a2  covariance      C = sum_i (x_i - mu)(x_i - mu)^T          (split over rows)
//   a5  JL correction   T = S P^T,  S Q = S - T P                 (small)
//   a6  embedding       Y = (X - mu) Pi^T  or  Y = X Pi^T         (n x r)
// One generic 64 x 64-tile kernel on v_mfma_f64_16x16x4f64: four waves, each
// a 32 x 32 block of 2 x 2 MFMA tiles, K staged through LDS in chunks of 16
// with the next chunk prefetched into registers.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace adg {

constexpr int GT = 64;   // output tile
constexpr int GK = 16;   // K chunk
constexpr int GPAD = 4;  // LDS row padding (doubles)

// ------------------------------------------------------------- operand views
// Element (m, k) of the left operand / (k, n) of the right operand.
struct CentredCols {      // A(m, k) = X[k][m] - mu[m]  (m = feature, k = point)
  const float* X; const double* mu; int64_t n, d;
  __device__ double operator()(int64_t m, int64_t k) const {
    return (m < d && k < n) ? (double)X[k * d + m] - mu[m] : 0.0;
  }
};
struct CentredColsB {     // B(k, n) = X[k][n] - mu[n]  (k = point, n = feature)
  const float* X; const double* mu; int64_t n, d;
  __device__ double operator()(int64_t k, int64_t c) const {
    return (c < d && k < n) ? (double)X[k * d + c] - mu[c] : 0.0;
  }
};
struct CentredRows {      // A(m, k) = X[m][k] - mu[k]  (m = point, k = feature); mu may be NULL
  const float* X; const double* mu; int64_t n, d;
  __device__ double operator()(int64_t m, int64_t k) const {
    if (m >= n || k >= d) return 0.0;
    double v = (double)X[m * d + k];
    return mu ? v - mu[k] : v;
  }
};
struct RowsF32T {         // B(k, n) = P[n][k] for an FP32 rows x cols matrix
  const float* P; int64_t rows, cols;
  __device__ double operator()(int64_t k, int64_t n) const {
    return (n < rows && k < cols) ? (double)P[n * cols + k] : 0.0;
  }
};
struct RowsF64 {          // A(m, k) = M[m][k]
  const double* M; int64_t rows, cols, ld;
  __device__ double operator()(int64_t m, int64_t k) const {
    return (m < rows && k < cols) ? M[m * ld + k] : 0.0;
  }
};
struct RowsF64T {         // B(k, n) = M[n][k]
  const double* M; int64_t rows, cols, ld;
  __device__ double operator()(int64_t k, int64_t n) const {
    return (n < rows && k < cols) ? M[n * ld + k] : 0.0;
  }
};
struct RowsF64N {         // B(k, n) = M[k][n]
  const double* M; int64_t rows, cols, ld;
  __device__ double operator()(int64_t k, int64_t n) const {
    return (k < rows && n < cols) ? M[k * ld + n] : 0.0;
  }
};

struct SketchSigns {       // A(a, i) = +-1/sqrt(m): top bit of SplitMix64 output (a << 32 | i) + 1
  uint64_t seed; int64_t m, n; double scale;
  __device__ double operator()(int64_t a, int64_t i) const {
    if (a >= m || i >= n) return 0.0;
    uint64_t z = seed + ((((uint64_t)a << 32) | (uint64_t)i) + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (z >> 63) ? -scale : scale;
  }
};

// ------------------------------------------------------------------ outputs
struct StoreF64 {         // C[m][n] (+ split offset)
  double* C; int64_t M, N, ld, split_stride;
  __device__ void operator()(int64_t m, int64_t n, int split, double v) const {
    if (m < M && n < N) C[split * split_stride + m * ld + n] = v;
  }
};
struct StoreF32 {
  float* C; int64_t M, N, ld;
  __device__ void operator()(int64_t m, int64_t n, int, double v) const {
    if (m < M && n < N) C[m * ld + n] = (float)v;
  }
};
struct StoreSQ {          // Pi[s + a][l] = fl32(S[a][l] - v), S from the sign matrix
  float* Pi; double* Pi64; const double* S; int64_t k, d, s;
  __device__ void operator()(int64_t a, int64_t l, int, double v) const {
    if (a < k && l < d) {
      double q = S[a * d + l] - v;
      Pi[(s + a) * d + l] = (float)q;
      if (Pi64) Pi64[(s + a) * d + l] = q;
    }
  }
};

__device__ inline void tri_tile(int64_t t, int64_t NT, int64_t& I, int64_t& J) {
  // Row-major enumeration of the upper triangle I <= J < NT: row I starts at
  // I*NT - I*(I-1)/2.
  double b = 2.0 * (double)NT + 1.0;
  int64_t i = (int64_t)((b - sqrt(b * b - 8.0 * (double)t)) * 0.5);
  if (i < 0) i = 0;
  if (i > NT - 1) i = NT - 1;
  while (i > 0 && i * NT - i * (i - 1) / 2 > t) --i;
  while (i + 1 < NT && (i + 1) * NT - (i + 1) * i / 2 <= t) ++i;
  I = i;
  J = i + (t - (i * NT - i * (i - 1) / 2));
}

// C(m, n) = sum_k A(m, k) B(k, n) over k in [k_begin, k_end) of this split.
// A_KC / B_KC: operand contiguous along k in memory (selects the coalesced
// thread mapping of the staging loads).  TRI: grid.x enumerates upper tiles.
template <class LA, class LB, class ST, bool A_KC, bool B_KC, bool TRI>
__global__ __launch_bounds__(256) void k_gemm64(LA la, LB lb, ST st, int64_t M, int64_t N, int64_t K,
                                                int64_t k_per_split, int64_t tiles_n) {
  __shared__ double As[2][GK][GT + GPAD];
  __shared__ double Bs[2][GK][GT + GPAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int64_t ti, tj;
  if (TRI) tri_tile(blockIdx.x, tiles_n, ti, tj);
  else { ti = blockIdx.x / tiles_n; tj = blockIdx.x % tiles_n; }
  const int64_t m0 = ti * GT, n0 = tj * GT;
  const int split = blockIdx.y;
  const int64_t kb = (int64_t)split * k_per_split;
  int64_t ke = kb + k_per_split;
  if (ke > K) ke = K;
  const int nch = ke > kb ? (int)((ke - kb + GK - 1) / GK) : 0;

  double ra[4], rb[4];
  auto fetch = [&](int c) {
    const int64_t k0 = kb + (int64_t)c * GK;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + u * 256;
      int kk, mm;
      if (A_KC) { kk = e % GK; mm = e / GK; } else { kk = e / GT; mm = e % GT; }
      const int64_t k = k0 + kk;
      ra[u] = k < ke ? la(m0 + mm, k) : 0.0;
      if (B_KC) { kk = e % GK; mm = e / GK; } else { kk = e / GT; mm = e % GT; }
      const int64_t k2 = k0 + kk;
      rb[u] = k2 < ke ? lb(k2, n0 + mm) : 0.0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + u * 256;
      int kk, mm;
      if (A_KC) { kk = e % GK; mm = e / GK; } else { kk = e / GT; mm = e % GT; }
      As[buf][kk][mm] = ra[u];
      if (B_KC) { kk = e % GK; mm = e / GK; } else { kk = e / GT; mm = e % GT; }
      Bs[buf][kk][mm] = rb[u];
    }
  };

  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (f64x4){0.0, 0.0, 0.0, 0.0};

  if (nch > 0) {
    fetch(0);
    stash(0);
    __syncthreads();
  }
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) fetch(c + 1);
#pragma unroll
    for (int ks = 0; ks < GK / 4; ++ks) {
      const int kr = ks * 4 + (lane >> 4);
      double a0 = As[buf][kr][wm * 32 + (lane & 15)];
      double a1 = As[buf][kr][wm * 32 + 16 + (lane & 15)];
      double b0 = Bs[buf][kr][wn * 32 + (lane & 15)];
      double b1 = Bs[buf][kr][wn * 32 + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (c + 1 < nch) stash(buf ^ 1);
    __syncthreads();
  }
  // D layout of v_mfma_f64_16x16x4f64: lane l, register v -> (4 v + l / 16, l % 16).
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + wm * 32 + a * 16 + 4 * v + (lane >> 4);
        const int64_t n = n0 + wn * 32 + b * 16 + (lane & 15);
        st(m, n, split, acc[a][b][v]);
      }
}

// Sum of the split partials of the upper tiles, mirrored to a full symmetric
// m_pad x m_pad matrix (zero outside d x d).
__global__ void k_cov_reduce(const double* __restrict__ part, int nsplit, int64_t d, int64_t m_pad,
                             double* __restrict__ C) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= m_pad * m_pad) return;
  const int64_t a = e / m_pad, b = e % m_pad;
  double s = 0.0;
  if (a < d && b < d) {
    const int64_t lo = a < b ? a : b, hi = a < b ? b : a;
    // upper tiles only: element (lo, hi) lives in tile (lo / GT, hi / GT) when
    // lo / GT <= hi / GT, which always holds for lo <= hi.
    for (int sp = 0; sp < nsplit; ++sp) s += part[(int64_t)sp * d * d + lo * d + hi];
  }
  C[e] = s;
}

// ---------------------------------------------------------------- launchers
hipError_t launch_cov_reduce(const double* part, int nsplit, int64_t d, int64_t m_pad, double* C, hipStream_t st) {
  k_cov_reduce<<<(unsigned)((m_pad * m_pad + 255) / 256), 256, 0, st>>>(part, nsplit, d, m_pad, C);
  return hipGetLastError();
}

hipError_t launch_covariance(const float* X, int64_t n, int64_t d, const double* mu, double* part,
                             int nsplit, double* C, int64_t m_pad, hipStream_t st) {
  const int64_t NT = (d + GT - 1) / GT;
  const int64_t ntiles = NT * (NT + 1) / 2;
  int64_t kps = round_up((n + nsplit - 1) / nsplit, GK);
  CentredCols A{X, mu, n, d};
  CentredColsB B{X, mu, n, d};
  StoreF64 S{part, d, d, d, d * d};
  dim3 g((unsigned)ntiles, (unsigned)nsplit);
  k_gemm64<CentredCols, CentredColsB, StoreF64, false, false, true><<<g, 256, 0, st>>>(A, B, S, d, d, n, kps, NT);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_cov_reduce<<<(unsigned)((m_pad * m_pad + 255) / 256), 256, 0, st>>>(part, nsplit, d, m_pad, C);
  return hipGetLastError();
}

// Y[i][c] = fl32(sum_l X[i][l] Pi[c][l])   (n x r, FP32)
hipError_t launch_embed_f32(const float* X, int64_t n, int64_t d, const float* Pi, int64_t r, float* Y,
                            hipStream_t st) {
  const int64_t tm = (n + GT - 1) / GT, tn = (r + GT - 1) / GT;
  CentredRows A{X, nullptr, n, d};
  RowsF32T B{Pi, r, d};
  StoreF32 S{Y, n, r, r};
  k_gemm64<CentredRows, RowsF32T, StoreF32, true, true, false><<<(unsigned)(tm * tn), 256, 0, st>>>(A, B, S, n, r, d, round_up(d, GK), tn);
  return hipGetLastError();
}

// T[a][b] = sum_l S[a][l] Vt[b][l]   (k x s)
hipError_t launch_proj_T(const double* S, int64_t k, int64_t d, const double* Vt, int64_t s, double* T,
                         hipStream_t st) {
  const int64_t tm = (k + GT - 1) / GT, tn = (s + GT - 1) / GT;
  RowsF64 A{S, k, d, d};
  RowsF64T B{Vt, s, d, d};
  StoreF64 Sv{T, k, s, s, 0};
  k_gemm64<RowsF64, RowsF64T, StoreF64, true, true, false><<<(unsigned)(tm * tn), 256, 0, st>>>(A, B, Sv, k, s, d, round_up(d, GK), tn);
  return hipGetLastError();
}

// Pi[s + a][l] = fl32(S[a][l] - sum_b T[a][b] Vt[b][l])   (k x d)
hipError_t launch_proj_SQ(const double* S, const double* T, int64_t k, int64_t s, const double* Vt,
                          int64_t d, float* Pi, double* Pi64, hipStream_t st) {
  const int64_t tm = (k + GT - 1) / GT, tn = (d + GT - 1) / GT;
  RowsF64 A{T, k, s, s};
  RowsF64N B{Vt, s, d, d};
  StoreSQ Sq{Pi, Pi64, S, k, d, s};
  k_gemm64<RowsF64, RowsF64N, StoreSQ, true, false, false><<<(unsigned)(tm * tn), 256, 0, st>>>(A, B, Sq, k, d, s, round_up(s > 0 ? s : 1, GK), tn);
  return hipGetLastError();
}

// Sum of split partials: out[e] = sum_s part[s * count + e].
__global__ void k_sum_splits(const double* __restrict__ part, int nsplit, int64_t count, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  double s = 0.0;
  for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * count + e];
  out[e] = s;
}

// C (M x N, row stride ldc) = A B^T with A (M x K, row stride lda) and B
// (N x K, row stride ldb), FP64.
hipError_t launch_gemm_nt(const double* A, int64_t M, int64_t K, int64_t lda, const double* B, int64_t N,
                          int64_t ldb, double* C, int64_t ldc, hipStream_t st) {
  const int64_t tm = (M + GT - 1) / GT, tn = (N + GT - 1) / GT;
  RowsF64 a{A, M, K, lda};
  RowsF64T b{B, N, K, ldb};
  StoreF64 c{C, M, N, ldc, 0};
  k_gemm64<RowsF64, RowsF64T, StoreF64, true, true, false><<<(unsigned)(tm * tn), 256, 0, st>>>(a, b, c, M, N, K, round_up(K, GK), tn);
  return hipGetLastError();
}

// C (M x N, row stride ldc) = A B with A (M x K, row stride lda) and B
// (K x N, row stride ldb), FP64.
hipError_t launch_gemm_nn(const double* A, int64_t M, int64_t K, int64_t lda, const double* B, int64_t N,
                          int64_t ldb, double* C, int64_t ldc, hipStream_t st) {
  const int64_t tm = (M + GT - 1) / GT, tn = (N + GT - 1) / GT;
  RowsF64 a{A, M, K, lda};
  RowsF64N b{B, K, N, ldb};
  StoreF64 c{C, M, N, ldc, 0};
  k_gemm64<RowsF64, RowsF64N, StoreF64, true, false, false><<<(unsigned)(tm * tn), 256, 0, st>>>(a, b, c, M, N, K, round_up(K, GK), tn);
  return hipGetLastError();
}

// Row i of Q (rows x cols) times lam_i^(-1/2), or 0 where lam_i <= rel lam_0
// (lam decreasing: directions the block does not span).
__global__ void k_scale_rows_isqrt(double* __restrict__ Q, int64_t rows, int64_t cols, const double* __restrict__ lam,
                                   double rel) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * cols) return;
  const double l = lam[e / cols];
  Q[e] = l > rel * lam[0] ? Q[e] / sqrt(l) : 0.0;
}
hipError_t launch_scale_rows_isqrt(double* Q, int64_t rows, int64_t cols, const double* lam, double rel,
                                   hipStream_t st) {
  k_scale_rows_isqrt<<<(unsigned)((rows * cols + 255) / 256), 256, 0, st>>>(Q, rows, cols, lam, rel);
  return hipGetLastError();
}

hipError_t launch_sketch(const float* X, int64_t n, int64_t d, const double* mu, int m, uint64_t sseed, double* part,
                         int nsplit, double* G, hipStream_t st) {
  const int64_t tm = (m + GT - 1) / GT, tn = (d + GT - 1) / GT;
  SketchSigns A{sseed, m, n, 1.0 / sqrt((double)m)};
  CentredColsB B{X, mu, n, d};
  StoreF64 S{part, m, d, d, (int64_t)m * d};
  const int64_t kps = round_up((n + nsplit - 1) / nsplit, GK);
  dim3 g((unsigned)(tm * tn), (unsigned)nsplit);
  k_gemm64<SketchSigns, CentredColsB, StoreF64, true, false, false><<<g, 256, 0, st>>>(A, B, S, m, d, n, kps, tn);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_sum_splits<<<(unsigned)((m * d + 255) / 256), 256, 0, st>>>(part, nsplit, (int64_t)m * d, G);
  return hipGetLastError();
}

hipError_t launch_gram_rows(const double* G, int m, int64_t d, double* K, int mp, hipStream_t st) {
  const int64_t tm = (mp + GT - 1) / GT;
  RowsF64 A{G, m, d, d};
  RowsF64T B{G, m, d, d};
  StoreF64 S{K, mp, mp, mp, 0};
  k_gemm64<RowsF64, RowsF64T, StoreF64, true, true, false><<<(unsigned)(tm * tm), 256, 0, st>>>(A, B, S, mp, mp, d, round_up(d, GK), tm);
  return hipGetLastError();
}

// Features of the learned search, from the sketch spectrum (decreasing lam):
//   f[i] = ln(sigma_i / ||sigma||_2 + 1e-6) / 4 for i < 64 (sigma = sqrt(lam)),
//   f[64] = ln(n) / 10, f[65] = ln(d) / 10, f[66] = 5 eps, f[67..79] = 0.
__global__ void k_sketch_features(const double* __restrict__ lam, int m, int64_t n, int64_t d, double eps,
                                  float* __restrict__ f) {
  if (threadIdx.x != 0) return;
  double tot = 0.0;
  for (int i = 0; i < m; ++i) tot += lam[i] > 0.0 ? lam[i] : 0.0;
  const double norm = sqrt(tot) > 0.0 ? sqrt(tot) : 1.0;
  for (int i = 0; i < 64; ++i) {
    const double sg = i < m && lam[i] > 0.0 ? sqrt(lam[i]) : 0.0;
    f[i] = (float)(log(sg / norm + 1e-6) / 4.0);
  }
  f[64] = (float)(log((double)n) / 10.0);
  f[65] = (float)(log((double)d) / 10.0);
  f[66] = (float)(5.0 * eps);
  for (int i = 67; i < 80; ++i) f[i] = 0.0f;
}

hipError_t launch_sketch_features(const double* lam, int m, int64_t n, int64_t d, double eps, float* feat,
                                  hipStream_t st) {
  k_sketch_features<<<1, 64, 0, st>>>(lam, m, n, d, eps, feat);
  return hipGetLastError();
}

}  // namespace adg
