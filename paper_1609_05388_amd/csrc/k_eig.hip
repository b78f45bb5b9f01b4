// Step a3 helpers: identity start of the eigenvector accumulator, the trace
// that scales the rotation threshold, and the final sort of the eigenpairs.
//
// The paper obtains P from an SVD (Sec. 2, PCA paragraph) through sklearn;
// the eigenvectors of C = Xc^T Xc are the same directions.  The eigensolver
// itself (block cyclic Jacobi: full FP64 accuracy for every eigenpair,
// including clustered and zero eigenvalues, with data-parallel steps) is in
// k_eig_block.hip.
#include "common.h"
#include "kernels.h"

namespace adg {

__global__ void k_eye(double* W, int m) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)m * m) return;
  W[e] = (e / m == e % m) ? 1.0 : 0.0;
}

// Sum of the diagonal (trace of a PSD matrix bounds its Frobenius norm).
__global__ void k_trace(const double* A, int m, double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) s += fabs(A[(int64_t)i * m + i]);
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// Sort eigenpairs by decreasing eigenvalue (ties: smaller index first) over
// the first d indices (index d of an odd-sized problem is padding).
// rank[a] = #{b < d : lam_b > lam_a or (lam_b == lam_a and b < a)}.
__global__ void k_eig_sort(const double* __restrict__ A, const double* __restrict__ W, int m, int d,
                           double* __restrict__ lam, double* __restrict__ Vt) {
  const int a = blockIdx.x;
  if (a >= d) return;
  __shared__ int rank_sh;
  __shared__ int cnt[256];
  const double la = A[(int64_t)a * m + a];
  int c = 0;
  for (int b = threadIdx.x; b < d; b += 256) {
    const double lb = A[(int64_t)b * m + b];
    c += (lb > la || (lb == la && b < a)) ? 1 : 0;
  }
  cnt[threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) cnt[threadIdx.x] += cnt[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) { rank_sh = cnt[0]; lam[cnt[0]] = la; }
  __syncthreads();
  const int rk = rank_sh;
  for (int l = threadIdx.x; l < d; l += 256) Vt[(int64_t)rk * d + l] = W[(int64_t)a * m + l];
}

// Constant coordinates: a coordinate whose centred values are all exactly
// zero has an all-zero row and column of C (every term of C_ij carries the
// factor x_i - mu_i = 0), so C is block diagonal with a zero block and its
// eigenpairs are those of the block of the other coordinates, embedded, plus
// eigenvalue 0 with the unit vectors of the constant coordinates.
// Eigenpairs of C from those of its non-constant block (lam1 decreasing,
// Vt1 rows, d1 of each; idx[0, d1) its coordinates, idx[d1, d) the constant
// ones) and eigenvalue 0 for each constant coordinate:
// element a < d1 is (lam1[a], Vt1[a] scattered to the coordinates idx[0, d1)),
// element a >= d1 is (0, unit vector of coordinate idx[a]); sorted by
// decreasing value, ties by a.  One workgroup per element.
__global__ void k_scatter_axes(const double* __restrict__ lam1, const double* __restrict__ Vt1,
                               const int* __restrict__ idx, int d1, int d, double* __restrict__ lam,
                               double* __restrict__ Vt) {
  const int a = blockIdx.x;
  if (a >= d) return;
  __shared__ int cnt[256];
  const double la = a < d1 ? lam1[a] : 0.0;
  int c = 0;
  for (int b = threadIdx.x; b < d; b += 256) {
    const double lb = b < d1 ? lam1[b] : 0.0;
    c += (lb > la || (lb == la && b < a)) ? 1 : 0;
  }
  cnt[threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) cnt[threadIdx.x] += cnt[threadIdx.x + o];
    __syncthreads();
  }
  const int rk = cnt[0];
  double* row = Vt + (int64_t)rk * d;
  for (int l = threadIdx.x; l < d; l += 256) row[l] = 0.0;
  __syncthreads();
  if (a < d1) {
    for (int c2 = threadIdx.x; c2 < d1; c2 += 256) row[idx[c2]] = Vt1[(int64_t)a * d1 + c2];
  } else if (threadIdx.x == 0) {
    row[idx[a]] = 1.0;
  }
  if (threadIdx.x == 0) lam[rk] = la;
}

// ---------------------------------------------------------------- launchers
hipError_t launch_scatter_axes(const double* lam1, const double* Vt1, const int* idx, int d1, int d, double* lam,
                               double* Vt, hipStream_t st) {
  k_scatter_axes<<<(unsigned)d, 256, 0, st>>>(lam1, Vt1, idx, d1, d, lam, Vt);
  return hipGetLastError();
}
hipError_t launch_eye(double* W, int m, hipStream_t st) {
  k_eye<<<(unsigned)(((int64_t)m * m + 255) / 256), 256, 0, st>>>(W, m);
  return hipGetLastError();
}
hipError_t launch_trace(const double* A, int m, double* out, hipStream_t st) {
  k_trace<<<1, 256, 0, st>>>(A, m, out);
  return hipGetLastError();
}
hipError_t launch_eig_sort(const double* A, const double* W, int m, int d, double* lam, double* Vt,
                           hipStream_t st) {
  k_eig_sort<<<(unsigned)d, 256, 0, st>>>(A, W, m, d, lam, Vt);
  return hipGetLastError();
}

}  // namespace adg
