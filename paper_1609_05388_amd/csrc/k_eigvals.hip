// Eigenvalues only of a small symmetric FP64 matrix (m <= 128), in one
// workgroup with the matrix resident in LDS: Householder reduction to
// tridiagonal form (Golub & Van Loan, Sec. 8.3.1), then every eigenvalue by
// bisection on Sturm sequence counts (Sec. 8.4.1), one thread per
// eigenvalue.  Used for the learned search's sketch spectrum, where the
// block Jacobi method (which also builds eigenvectors) costs far more than
// the whole rest of the feature computation.
#include "common.h"
#include "kernels.h"

namespace adg {

constexpr int EVM = 128;        // largest supported m
constexpr int EVLD = EVM + 1;   // LDS row stride (doubles)

__device__ inline double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// Number of eigenvalues of the tridiagonal (d, e) below x (Sturm count of
// the LDL^T pivots q_k = d_k - x - e_{k-1}^2 / q_{k-1}; a zero pivot is
// replaced by a tiny negative number).
__device__ inline int sturm_count(const double* d, const double* e2, int m, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  c += q < 0.0;
  for (int k = 1; k < m; ++k) {
    q = d[k] - x - e2[k - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

// A: m x m (row stride lda), symmetric.  lam: m eigenvalues, decreasing.
__global__ __launch_bounds__(256) void k_sym_eigvals(const double* __restrict__ A, int m, int lda,
                                                     double* __restrict__ lam) {
  extern __shared__ double ev_lds[];
  double* S = ev_lds;                 // [EVM][EVLD]
  double* v = S + EVM * EVLD;         // Householder vector
  double* p = v + EVM;                // p, then w
  double* dd = p + EVM;               // diagonal
  double* ee = dd + EVM;              // squared off-diagonal
  double* red = ee + EVM;             // 4 partial sums + scalars
  const int tid = threadIdx.x;
  for (int e = tid; e < m * m; e += 256) S[(e / m) * EVLD + (e % m)] = A[(int64_t)(e / m) * lda + (e % m)];
  __syncthreads();

  // Householder: column k below the diagonal -> (alpha, 0, ..., 0)
  for (int k = 0; k + 2 < m; ++k) {
    const int n = m - k - 1;          // trailing size
    double x = 0.0;
    if (tid < n) {
      x = S[(k + 1 + tid) * EVLD + k];
      v[tid] = x;
    }
    const double nrm2 = block_sum(tid < n ? x * x : 0.0, red);
    const double x0 = S[(k + 1) * EVLD + k];
    const double tail = nrm2 - x0 * x0;
    if (tail <= 0.0) {                // already tridiagonal in this column
      if (tid == 0) { dd[k] = S[k * EVLD + k]; ee[k] = x0 * x0; }
      __syncthreads();
      continue;
    }
    const double alpha = x0 >= 0.0 ? -sqrt(nrm2) : sqrt(nrm2);
    const double v0 = x0 - alpha;
    const double vtv = tail + v0 * v0;
    const double beta = 2.0 / vtv;
    if (tid == 0) {
      v[0] = v0;
      dd[k] = S[k * EVLD + k];
      ee[k] = alpha * alpha;
    }
    __syncthreads();
    // p = beta A' v  (A' = trailing n x n block)
    double pi = 0.0;
    if (tid < n) {
      const double* row = S + (k + 1 + tid) * EVLD + (k + 1);
      for (int j = 0; j < n; ++j) pi = fma(row[j], v[j], pi);
      pi *= beta;
    }
    const double pv = block_sum(tid < n ? pi * v[tid] : 0.0, red);
    // w = p - (beta p^T v / 2) v
    if (tid < n) p[tid] = pi - 0.5 * beta * pv * v[tid];
    __syncthreads();
    // A' -= v w^T + w v^T
    for (int e = tid; e < n * n; e += 256) {
      const int i = e / n, j = e % n;
      double* a = S + (k + 1 + i) * EVLD + (k + 1 + j);
      *a = *a - v[i] * p[j] - p[i] * v[j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (m >= 2) {
      dd[m - 2] = S[(m - 2) * EVLD + (m - 2)];
      const double t = S[(m - 1) * EVLD + (m - 2)];
      ee[m - 2] = t * t;
    }
    dd[m - 1] = S[(m - 1) * EVLD + (m - 1)];
  }
  __syncthreads();

  // Gershgorin interval and bisection: thread i finds the eigenvalue of rank
  // m - 1 - i from below (the i-th largest).
  if (tid < m) {
    double lo = 0.0, hi = 0.0, scale = 0.0;
    for (int k = 0; k < m; ++k) {
      const double r = (k > 0 ? sqrt(ee[k - 1]) : 0.0) + (k + 1 < m ? sqrt(ee[k]) : 0.0);
      lo = k == 0 ? dd[k] - r : fmin(lo, dd[k] - r);
      hi = k == 0 ? dd[k] + r : fmax(hi, dd[k] + r);
      scale = fmax(scale, fabs(dd[k]) + r);
    }
    const double pivmin = fmax(scale, 1e-300) * 1e-300;
    const int want = m - 1 - tid;     // number of eigenvalues strictly below the target
    double a = lo - 1e-12 * scale - 1e-300, b = hi + 1e-12 * scale + 1e-300;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (a + b);
      if (mid <= a || mid >= b) break;
      if (b - a <= 2.0 * kU64 * scale) break;
      if (sturm_count(dd, ee, m, mid, pivmin) > want) b = mid;
      else a = mid;
    }
    lam[tid] = 0.5 * (a + b);
  }
}

constexpr size_t kLdsEigvals = (EVM * EVLD + 4 * EVM + 8) * sizeof(double);

hipError_t launch_sym_eigvals(const double* A, int m, int lda, double* lam, hipStream_t st) {
  if (m < 1 || m > EVM) return hipErrorInvalidValue;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sym_eigvals),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsEigvals);
    if (e != hipSuccess) return e;
    attr = true;
  }
  k_sym_eigvals<<<1, 256, kLdsEigvals, st>>>(A, m, lda, lam);
  return hipGetLastError();
}

}  // namespace adg
