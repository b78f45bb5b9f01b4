// Step a1: mean row, centring, row norms and per-row bound terms.
//
// The paper's PCA works on zero-centred data (Sec. 2, PCA paragraph, eq. 4).
// Distances are translation invariant, so the all-pairs screen also works on
// centred rows: it shrinks ||x||^2 + ||y||^2 - 2 x.y cancellation.
#include "common.h"
#include "kernels.h"

namespace adg {

// Partial column sums over a chunk of rows (FP64), plus a non-finite flag.
// grid (ceil(m / 256), nchunks), block 256: thread = one column.
template <typename T>
__global__ void k_colsum_partial(const T* __restrict__ A, int64_t n, int64_t m, int64_t ld,
                                 int64_t rows_per_chunk, double* __restrict__ partial,
                                 int* __restrict__ nonfinite) {
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= m) return;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < n ? r0 + rows_per_chunk : n;
  double s = 0.0;
  int bad = 0;
  for (int64_t i = r0; i < r1; ++i) {
    const double v = (double)A[i * ld + col];
    bad |= !isfinite(v);
    s += v;
  }
  partial[(int64_t)blockIdx.y * m + col] = s;
  if (bad) atomicOr(nonfinite, 1);
}

// mu[col] = (sum over chunks, in chunk order) / n.
__global__ void k_colsum_final(const double* __restrict__ partial, int64_t nchunks, int64_t m,
                               int64_t n, double* __restrict__ mu) {
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= m) return;
  double s = 0.0;
  for (int64_t c = 0; c < nchunks; ++c) s += partial[c * m + col];
  mu[col] = s / (double)n;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Centred FP32 copy of rows: dst[i][l] = fl32(src[i][l] - mu[l]) for i < n,
// l < m; zero in the padding (l in [m, ldd), i in [n, n_pad)).  mu may be
// NULL (rows already centred).  norm2[i] = ||dst_i||^2 in FP64.
// One wave per row, 4 rows per block of 256.
template <typename T>
__global__ void k_center_rows(const T* __restrict__ src, int64_t n, int64_t m, int64_t lds,
                              const double* __restrict__ mu, float* __restrict__ dst, int64_t ldd,
                              int64_t n_pad, double* __restrict__ norm2) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n_pad) return;
  double s = 0.0;
  for (int64_t l = lane; l < ldd; l += 64) {
    float v = 0.0f;
    if (row < n && l < m) {
      double c = (double)src[row * lds + l];
      if (mu) c -= mu[l];
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

// ---------------------------------------------------------------- launchers
template <typename T>
hipError_t launch_mean(const T* A, int64_t n, int64_t m, int64_t ld, double* partial,
                       int64_t nchunks, int64_t rows_per_chunk, double* mu, int* nonfinite,
                       hipStream_t st) {
  dim3 g((unsigned)((m + 255) / 256), (unsigned)nchunks);
  k_colsum_partial<T><<<g, 256, 0, st>>>(A, n, m, ld, rows_per_chunk, partial, nonfinite);
  k_colsum_final<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(partial, nchunks, m, n, mu);
  return hipGetLastError();
}
template hipError_t launch_mean<float>(const float*, int64_t, int64_t, int64_t, double*, int64_t,
                                       int64_t, double*, int*, hipStream_t);

template <typename T>
hipError_t launch_center(const T* src, int64_t n, int64_t m, int64_t lds, const double* mu,
                         float* dst, int64_t ldd, int64_t n_pad, double* norm2, hipStream_t st) {
  k_center_rows<T><<<(unsigned)((n_pad + 3) / 4), 256, 0, st>>>(src, n, m, lds, mu, dst, ldd, n_pad, norm2);
  return hipGetLastError();
}
template hipError_t launch_center<float>(const float*, int64_t, int64_t, int64_t, const double*,
                                         float*, int64_t, int64_t, double*, hipStream_t);
template hipError_t launch_center<double>(const double*, int64_t, int64_t, int64_t, const double*,
                                          float*, int64_t, int64_t, double*, hipStream_t);

hipError_t launch_row_terms(const double* norm2, double c_self, const double* norm2_other,
                            double c_other, int64_t n_pad, float2* terms, hipStream_t st) {
  k_row_terms<<<(unsigned)((n_pad + 255) / 256), 256, 0, st>>>(norm2, c_self, norm2_other, c_other, n_pad, terms);
  return hipGetLastError();
}

}  // namespace adg
