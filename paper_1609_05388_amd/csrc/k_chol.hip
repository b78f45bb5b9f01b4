// Cholesky factor for the screen images of a map with more rows than the
// cloud has non-constant coordinates.
//
// For a map Pi (r x d) and a pair difference v (non-constant coordinates
// only, d' of them), ||Pi v||^2 = v^T M v with M = Pi'^T Pi' (d' x d'; Pi' the
// columns of Pi at those coordinates).  When r > d', the factor M = L L^T
// gives images z = L^T x of d' coordinates whose distances are the map's:
// the all-pairs screen then runs over d' image columns instead of r.
//
// One workgroup, blocked right-looking: for each panel of 32 columns the
// panel (rows j0..m-1) is factored in LDS, written back, and the trailing
// lower triangle is updated with the panel's outer products.  Every entry of
// L is an ordinary Cholesky entry, (a_ij - sum_k l_ik l_jk) / l_jj, with the
// sum taken in some order, so the computed factor satisfies the textbook
// backward error bound L L^T = M + E, |E| <= gamma_{m+1} |L| |L^T|, for any
// order of the sums.
#include "common.h"
#include "kernels.h"

namespace adg {

constexpr int CB = 32;           // panel width
constexpr int kCholMaxM = 600;   // LDS panel: kCholMaxM x CB doubles

// A: m x m FP64, column-major (ld m), symmetric positive definite; on return
// its lower triangle holds L (A = L L^T) and its strict upper triangle zero.
// *fail = 1 (set, never cleared) on a pivot that is not positive and finite.
__global__ __launch_bounds__(1024) void k_cholesky(double* __restrict__ A, int m, int* __restrict__ fail) {
  __shared__ double P[kCholMaxM * CB];   // panel, P[(i - j0) + c * rows]
  __shared__ double piv;
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  __syncthreads();
  for (int j0 = 0; j0 < m; j0 += CB) {
    const int nb = min(CB, m - j0), rows = m - j0;
    for (int e = t; e < rows * nb; e += 1024) {
      const int c = e / rows, i = e - c * rows;
      P[e] = A[(int64_t)(j0 + c) * m + j0 + i];
    }
    __syncthreads();
    // factor the panel in LDS
    for (int c = 0; c < nb; ++c) {
      if (t == 0) {
        const double a = P[c + c * rows];
        if (!(a > 0.0) || !isfinite(a)) {
          bad = 1;
          piv = 1.0;
        } else {
          piv = sqrt(a);
        }
        P[c + c * rows] = piv;
      }
      __syncthreads();
      if (bad) break;   // uniform: every thread reads it after the barrier
      for (int i = c + 1 + t; i < rows; i += 1024) P[i + c * rows] /= piv;
      __syncthreads();
      // panel columns c + 1 .. nb - 1, rows at or below the diagonal
      const int w = nb - c - 1;
      for (int e = t; e < w * rows; e += 1024) {
        const int cc = c + 1 + e / rows, i = e - (e / rows) * rows;
        if (i >= cc) P[i + cc * rows] -= P[i + c * rows] * P[cc + c * rows];
      }
      __syncthreads();
    }
    if (bad) break;
    for (int e = t; e < rows * nb; e += 1024) {
      const int c = e / rows, i = e - c * rows;
      A[(int64_t)(j0 + c) * m + j0 + i] = P[e];
    }
    // trailing lower triangle: columns k and rows i >= k past the panel
    const int w = rows - nb;
    for (int64_t e = t; e < (int64_t)w * w; e += 1024) {
      const int kc = (int)(e / w), ir = (int)(e - (int64_t)kc * w);
      if (ir < kc) continue;
      const int pi = nb + ir, pk = nb + kc;   // panel rows of i and k
      double s = 0.0;
      for (int c = 0; c < nb; ++c) s = fma(P[pi + c * rows], P[pk + c * rows], s);
      A[(int64_t)(j0 + nb + kc) * m + j0 + nb + ir] -= s;
    }
    __syncthreads();
  }
  for (int64_t e = t; e < (int64_t)m * m; e += 1024) {
    const int64_t c = e / m, r = e - c * m;
    if (r < c) A[e] = 0.0;
  }
  if (t == 0 && bad) *fail = 1;
}

int chol_max_m() { return kCholMaxM; }

hipError_t launch_cholesky(double* A, int m, int* fail, hipStream_t st) {
  if (m < 1 || m > kCholMaxM) return hipErrorInvalidValue;
  k_cholesky<<<1, 1024, 0, st>>>(A, m, fail);
  return hipGetLastError();
}

}  // namespace adg
