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
// Per panel column: every thread takes the pivot from the diagonal (the same
// value for all, so the exit on a bad pivot is uniform), the scaled column
// goes to lc, then the panel's later columns are updated from lc (two
// barriers per column).  The trailing update gives each thread four rows of
// one column, so a panel value of that column serves four products.
__global__ __launch_bounds__(1024) void k_cholesky(double* __restrict__ A, int m, int* __restrict__ fail) {
  __shared__ double P[kCholMaxM * CB];   // panel, P[(i - j0) + c * rows]
  __shared__ double lc[kCholMaxM];       // the current panel column, scaled
  const int t = threadIdx.x;
  bool bad = false;
  for (int j0 = 0; j0 < m && !bad; j0 += CB) {
    const int nb = min(CB, m - j0), rows = m - j0;
    for (int e = t; e < rows * nb; e += 1024) {
      const int c = e / rows, i = e - c * rows;
      P[e] = A[(int64_t)(j0 + c) * m + j0 + i];
    }
    __syncthreads();
    for (int c = 0; c < nb; ++c) {
      const double a = P[c + c * rows];
      if (!(a > 0.0) || !isfinite(a)) {   // the same value in every thread
        bad = true;
        break;
      }
      const double piv = sqrt(a);
      for (int i = c + t; i < rows; i += 1024) lc[i] = i == c ? piv : P[i + c * rows] / piv;
      __syncthreads();
      for (int i = c + t; i < rows; i += 1024) P[i + c * rows] = lc[i];
      const int w = nb - c - 1;
      for (int e = t; e < w * rows; e += 1024) {
        const int cc = c + 1 + e / rows, i = e - (e / rows) * rows;
        if (i >= cc) P[i + cc * rows] -= lc[i] * lc[cc];
      }
      __syncthreads();
    }
    if (bad) break;
    for (int e = t; e < rows * nb; e += 1024) {
      const int c = e / rows, i = e - c * rows;
      A[(int64_t)(j0 + c) * m + j0 + i] = P[e];
    }
    // trailing lower triangle: column kc, rows 4 q .. 4 q + 3 (those >= kc)
    const int w = rows - nb, wq = (w + 3) / 4;
    for (int64_t e = t; e < (int64_t)w * wq; e += 1024) {
      const int kc = (int)(e / wq), i0 = 4 * (int)(e - (int64_t)kc * wq);
      if (i0 + 3 < kc) continue;
      const int pk = nb + kc;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      const bool v1 = i0 + 1 < w, v2 = i0 + 2 < w, v3 = i0 + 3 < w;
      for (int c = 0; c < nb; ++c) {
        const double* col = P + c * rows + nb + i0;
        const double bk = P[pk + c * rows];
        s0 = fma(col[0], bk, s0);
        if (v1) s1 = fma(col[1], bk, s1);
        if (v2) s2 = fma(col[2], bk, s2);
        if (v3) s3 = fma(col[3], bk, s3);
      }
      double* out = A + (int64_t)(j0 + nb + kc) * m + j0 + nb + i0;
      if (i0 >= kc) out[0] -= s0;
      if (v1 && i0 + 1 >= kc) out[1] -= s1;
      if (v2 && i0 + 2 >= kc) out[2] -= s2;
      if (v3 && i0 + 3 >= kc) out[3] -= s3;
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
