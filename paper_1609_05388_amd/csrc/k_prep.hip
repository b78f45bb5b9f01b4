// Step a1: mean row, centring, row norms and per-row bound terms.
//
// The paper's PCA works on zero-centred data (Sec. 2, PCA paragraph, eq. 4).
// Distances are translation invariant, so the all-pairs screen also works on
// centred rows: it shrinks ||x||^2 + ||y||^2 - 2 x.y cancellation.
#include "common.h"
#include "kernels.h"

namespace adg {

// Partial column sums over a chunk of rows (FP64), plus a non-finite flag
// and, when pmin is given, the chunk's smallest and largest value.
// grid (ceil(m / 256), nchunks), block 256: thread = one column.
template <typename T>
__global__ void k_colsum_partial(const T* __restrict__ A, int64_t n, int64_t m, int64_t ld,
                                 int64_t rows_per_chunk, double* __restrict__ partial,
                                 int* __restrict__ nonfinite, double* __restrict__ pmin,
                                 double* __restrict__ pmax) {
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= m) return;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < n ? r0 + rows_per_chunk : n;
  double s = 0.0, lo = INFINITY, hi = -INFINITY;
  int bad = 0;
  for (int64_t i = r0; i < r1; ++i) {
    const double v = (double)A[i * ld + col];
    bad |= !isfinite(v);
    s += v;
    lo = fmin(lo, v);
    hi = fmax(hi, v);
  }
  partial[(int64_t)blockIdx.y * m + col] = s;
  if (pmin) {
    pmin[(int64_t)blockIdx.y * m + col] = lo;
    pmax[(int64_t)blockIdx.y * m + col] = hi;
  }
  if (bad) atomicOr(nonfinite, 1);
}

// mu[col] = (sum over chunks, in chunk order) / n.  With pmin, keep[col] = 1
// unless the column holds one value only.  Such a column's mean is exactly
// that value (n < 2^29 copies of an FP32 value sum exactly in FP64), so its
// centred entries are exactly zero.
__global__ void k_colsum_final(const double* __restrict__ partial, int64_t nchunks, int64_t m,
                               int64_t n, double* __restrict__ mu, const double* __restrict__ pmin,
                               const double* __restrict__ pmax, int* __restrict__ keep) {
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= m) return;
  double s = 0.0, lo = INFINITY, hi = -INFINITY;
  for (int64_t c = 0; c < nchunks; ++c) {
    s += partial[c * m + col];
    if (pmin) {
      lo = fmin(lo, pmin[c * m + col]);
      hi = fmax(hi, pmax[c * m + col]);
    }
  }
  mu[col] = s / (double)n;
  if (pmin) keep[col] = (lo != hi || n >= ((int64_t)1 << 29)) ? 1 : 0;
}

// Stable compaction of m flags (one workgroup): idx[0, k) = the indices with
// keep = 1 ascending, idx[k, m) the others ascending; *k_out = k.
__global__ __launch_bounds__(1024) void k_compact_keep(const int* __restrict__ keep, int m, int* __restrict__ idx,
                                                       int* __restrict__ k_out) {
  __shared__ int wsum[2][16];
  __shared__ int base[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) { base[0] = 0; base[1] = 0; }
  int nk = 0;
  for (int i = tid; i < m; i += 1024) nk += keep[i] ? 1 : 0;
  for (int o = 32; o >= 1; o >>= 1) nk += __shfl_xor(nk, o, 64);
  if (lane == 0) wsum[0][wave] = nk;
  __syncthreads();
  int k = 0;
  for (int w = 0; w < 16; ++w) k += wsum[0][w];
  __syncthreads();
  for (int c0 = 0; c0 < m; c0 += 1024) {
    const int i = c0 + tid;
    const bool in = i < m;
    const bool kp = in && keep[i];
    const uint64_t bk = __builtin_amdgcn_ballot_w64(kp);
    const uint64_t bz = __builtin_amdgcn_ballot_w64(in && !kp);
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    if (lane == 0) { wsum[0][wave] = __popcll(bk); wsum[1][wave] = __popcll(bz); }
    __syncthreads();
    int ok = base[0], oz = base[1];
    for (int w = 0; w < wave; ++w) { ok += wsum[0][w]; oz += wsum[1][w]; }
    if (kp) idx[ok + __popcll(bk & below)] = i;
    else if (in) idx[k + oz + __popcll(bz & below)] = i;
    __syncthreads();
    if (tid == 0) {
      for (int w = 0; w < 16; ++w) { base[0] += wsum[0][w]; base[1] += wsum[1][w]; }
    }
    __syncthreads();
  }
  if (tid == 0) *k_out = k;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Centred FP32 copy of rows: dst[i][l] = fl32(src[i][c] - mu[c]) with
// c = colmap[l] (c = l without a map) for i < n, l < m; zero in the padding
// (l in [m, ldd), i in [n, n_pad)).  mu may be NULL (rows already centred).
// norm2[i] = ||dst_i||^2 in FP64.  One wave per row, 4 rows per block of 256.
template <typename T>
__global__ void k_center_rows(const T* __restrict__ src, int64_t n, int64_t m, int64_t lds,
                              const double* __restrict__ mu, float* __restrict__ dst, int64_t ldd,
                              int64_t n_pad, double* __restrict__ norm2, const int* __restrict__ colmap) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n_pad) return;
  double s = 0.0;
  for (int64_t l = lane; l < ldd; l += 64) {
    float v = 0.0f;
    if (row < n && l < m) {
      const int64_t c0 = colmap ? colmap[l] : l;
      double c = (double)src[row * lds + c0];
      if (mu) c -= mu[c0];
      v = (float)c;
    }
    dst[row * ldd + l] = v;
    s += (double)v * (double)v;
  }
  s = wave_sum(s);
  if (lane == 0) norm2[row] = s;
}

__device__ inline float f32_down(double x) {
  float f = (float)x;
  if ((double)f > x) f = nextafterf(f, -INFINITY);
  return f;
}
__device__ inline float f32_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = nextafterf(f, INFINITY);
  return f;
}

// Per-row bound terms of the screen: with N the row's own squared norm and
// N' a second norm (may be NULL),
//   lo = N - c_self * N - c_other * N'   (rounded down to FP32),
//   hi = N + c_self * N + c_other * N'   (rounded up to FP32).
// The screen forms D^2 bounds as (lo_i + lo_j) - 2 g and (hi_i + hi_j) - 2 g.
__global__ void k_row_terms(const double* __restrict__ norm2, double c_self,
                            const double* __restrict__ norm2_other, double c_other,
                            int64_t n_pad, float2* __restrict__ terms) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n_pad) return;
  const double N = norm2[i];
  const double slack = c_self * N + (norm2_other ? c_other * norm2_other[i] : 0.0);
  terms[i] = make_float2(f32_down(N - slack), f32_up(N + slack));
}

// FP64 centred copy of the listed columns: dst[i][c] = src[i][k] - mu[k],
// k = colmap[c] (FP64 difference of the FP32 value), n x m row-major.
__global__ void k_center64(const float* __restrict__ src, int64_t n, int64_t lds, const double* __restrict__ mu,
                           const int* __restrict__ colmap, int64_t m, double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * m) return;
  const int64_t i = e / m, c = e % m;
  const int64_t k = colmap[c];
  dst[e] = (double)src[i * lds + k] - mu[k];
}

// FP64 copy of the listed columns of an FP32 r x d map (exact): r x m.
__global__ void k_cols64(const float* __restrict__ P, int64_t r, int64_t d, const int* __restrict__ colmap, int64_t m,
                         double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= r * m) return;
  const int64_t j = e / m, c = e % m;
  dst[e] = (double)P[j * d + colmap[c]];
}

// ---------------------------------------------------------------- launchers
hipError_t launch_center64(const float* src, int64_t n, int64_t lds, const double* mu, const int* colmap, int64_t m,
                           double* dst, hipStream_t st) {
  k_center64<<<(unsigned)((n * m + 255) / 256), 256, 0, st>>>(src, n, lds, mu, colmap, m, dst);
  return hipGetLastError();
}
hipError_t launch_cols64(const float* P, int64_t r, int64_t d, const int* colmap, int64_t m, double* dst,
                         hipStream_t st) {
  k_cols64<<<(unsigned)((r * m + 255) / 256), 256, 0, st>>>(P, r, d, colmap, m, dst);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_mean(const T* A, int64_t n, int64_t m, int64_t ld, double* partial,
                       int64_t nchunks, int64_t rows_per_chunk, double* mu, int* nonfinite,
                       hipStream_t st, double* pmin, double* pmax, int* keep) {
  dim3 g((unsigned)((m + 255) / 256), (unsigned)nchunks);
  k_colsum_partial<T><<<g, 256, 0, st>>>(A, n, m, ld, rows_per_chunk, partial, nonfinite, pmin, pmax);
  k_colsum_final<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(partial, nchunks, m, n, mu, pmin, pmax, keep);
  return hipGetLastError();
}
template hipError_t launch_mean<float>(const float*, int64_t, int64_t, int64_t, double*, int64_t,
                                       int64_t, double*, int*, hipStream_t, double*, double*, int*);

hipError_t launch_compact_keep(const int* keep, int m, int* idx, int* k_out, hipStream_t st) {
  k_compact_keep<<<1, 1024, 0, st>>>(keep, m, idx, k_out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_center(const T* src, int64_t n, int64_t m, int64_t lds, const double* mu,
                         float* dst, int64_t ldd, int64_t n_pad, double* norm2, hipStream_t st,
                         const int* colmap) {
  k_center_rows<T><<<(unsigned)((n_pad + 3) / 4), 256, 0, st>>>(src, n, m, lds, mu, dst, ldd, n_pad, norm2,
                                                                 colmap);
  return hipGetLastError();
}
template hipError_t launch_center<float>(const float*, int64_t, int64_t, int64_t, const double*,
                                         float*, int64_t, int64_t, double*, hipStream_t, const int*);
template hipError_t launch_center<double>(const double*, int64_t, int64_t, int64_t, const double*,
                                          float*, int64_t, int64_t, double*, hipStream_t, const int*);

hipError_t launch_row_terms(const double* norm2, double c_self, const double* norm2_other,
                            double c_other, int64_t n_pad, float2* terms, hipStream_t st) {
  k_row_terms<<<(unsigned)((n_pad + 255) / 256), 256, 0, st>>>(norm2, c_self, norm2_other, c_other, n_pad, terms);
  return hipGetLastError();
}

}  // namespace adg
