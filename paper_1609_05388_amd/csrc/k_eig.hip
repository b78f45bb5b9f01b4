// Step a3: eigenpairs of the FP64 covariance by the parallel cyclic Jacobi
// method (two-sided rotations, round-robin "chess tournament" ordering: in
// each of the m - 1 rounds of a sweep the m indices form m / 2 disjoint
// pairs, so all m / 2 rotations of a round commute and run at once).
//
// The paper obtains P from an SVD (Sec. 2, PCA paragraph) through sklearn;
// the eigenvectors of C = Xc^T Xc are the same directions.  Jacobi is used
// because it converges to full FP64 accuracy for every eigenpair, including
// clustered and zero eigenvalues, with only data-parallel steps.
//
// One launch per round updates A' = J^T A J into a second buffer (each thread
// owns one 2 x 2 block {p_a, q_a} x {p_b, q_b}) and rotates the rows of
// W = V^T (row i of W becomes eigenvector i).
#include "common.h"
#include "kernels.h"

namespace adg {

// Pair k (0 <= k < m/2) of round t for m players (m even), M = m - 1:
// k = 0 pairs player 0 with (t mod M) + 1; k >= 1 pairs (t + k) mod M + 1 with
// (t - k) mod M + 1.  Returned as p < q.
__device__ inline void rr_pair(int t, int k, int m, int& p, int& q) {
  const int M = m - 1;
  int a, b;
  if (k == 0) { a = 0; b = t % M + 1; }
  else { a = (t + k) % M + 1; b = ((t - k) % M + M) % M + 1; }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// Rotation (c, s) annihilating A[p][q] (Golub & Van Loan, sym.schur2):
// tau = (A_qq - A_pp) / (2 A_pq), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
// c = 1 / sqrt(1 + t^2), s = t c; J has J_pp = J_qq = c, J_pq = s, J_qp = -s.
// Skipped (c = 1, s = 0) when |A_pq| <= thr.
__device__ inline bool rotation(const double* A, int m, int p, int q, double thr, double& c, double& s,
                                double& t) {
  const double apq = A[(int64_t)p * m + q];
  if (!(fabs(apq) > thr)) { c = 1.0; s = 0.0; t = 0.0; return false; }
  const double app = A[(int64_t)p * m + p], aqq = A[(int64_t)q * m + q];
  const double tau = (aqq - app) / (2.0 * apq);
  if (fabs(tau) > 1e150) t = 0.5 / tau;
  else t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
  return true;
}

constexpr int EB = 16;  // pairs per block side

// Grid: blocks [0, nA) update A (EB x EB pair blocks), blocks [nA, nA + nW)
// rotate W rows (EB pairs x 16 columns each).
__global__ __launch_bounds__(256) void k_jacobi_round(const double* __restrict__ A, double* __restrict__ A2,
                                                      double* __restrict__ W, int m, int t, double thr,
                                                      int nA, int* __restrict__ rot_count) {
  __shared__ double cs_r[EB][2], cs_c[EB][2], tt[EB];
  __shared__ int pr[EB][2], pc[EB][2];
  const int half = m / 2;
  const int gb = (half + EB - 1) / EB;
  const int tid = threadIdx.x;
  if ((int)blockIdx.x < nA) {
    const int br = blockIdx.x / gb, bc = blockIdx.x % gb;
    if (tid < 2 * EB) {
      const int side = tid / EB, u = tid % EB;
      const int k = (side == 0 ? br : bc) * EB + u;
      if (k < half) {
        int p, q;
        rr_pair(t, k, m, p, q);
        double c, s, tv;
        rotation(A, m, p, q, thr, c, s, tv);
        if (side == 0) { cs_r[u][0] = c; cs_r[u][1] = s; pr[u][0] = p; pr[u][1] = q; tt[u] = tv; }
        else { cs_c[u][0] = c; cs_c[u][1] = s; pc[u][0] = p; pc[u][1] = q; }
      }
    }
    __syncthreads();
    const int ur = tid / EB, uc = tid % EB;
    const int ka = br * EB + ur, kb = bc * EB + uc;
    if (ka >= half || kb >= half) return;
    const int pa = pr[ur][0], qa = pr[ur][1], pb = pc[uc][0], qb = pc[uc][1];
    const double ca = cs_r[ur][0], sa = cs_r[ur][1], cb = cs_c[uc][0], sb = cs_c[uc][1];
    if (ka == kb) {
      const double app = A[(int64_t)pa * m + pa], aqq = A[(int64_t)qa * m + qa], apq = A[(int64_t)pa * m + qa];
      const double tv = tt[ur];
      A2[(int64_t)pa * m + pa] = app - tv * apq;
      A2[(int64_t)qa * m + qa] = aqq + tv * apq;
      A2[(int64_t)pa * m + qa] = sa != 0.0 ? 0.0 : apq;
      A2[(int64_t)qa * m + pa] = sa != 0.0 ? 0.0 : apq;
      return;
    }
    const double m00 = A[(int64_t)pa * m + pb], m01 = A[(int64_t)pa * m + qb];
    const double m10 = A[(int64_t)qa * m + pb], m11 = A[(int64_t)qa * m + qb];
    // rows: new row p = c A_p - s A_q, new row q = s A_p + c A_q
    const double r00 = ca * m00 - sa * m10, r01 = ca * m01 - sa * m11;
    const double r10 = sa * m00 + ca * m10, r11 = sa * m01 + ca * m11;
    // columns: new col p = c col_p - s col_q, new col q = s col_p + c col_q
    A2[(int64_t)pa * m + pb] = cb * r00 - sb * r01;
    A2[(int64_t)pa * m + qb] = sb * r00 + cb * r01;
    A2[(int64_t)qa * m + pb] = cb * r10 - sb * r11;
    A2[(int64_t)qa * m + qb] = sb * r10 + cb * r11;
  } else {
    const int wb = blockIdx.x - nA;
    const int ncol16 = (m + 15) / 16;
    const int bp = wb / ncol16, bcol = wb % ncol16;
    if (tid < EB) {
      const int k = bp * EB + tid;
      if (k < half) {
        int p, q;
        rr_pair(t, k, m, p, q);
        double c, s, tv;
        const bool applied = rotation(A, m, p, q, thr, c, s, tv);
        cs_r[tid][0] = c; cs_r[tid][1] = s; pr[tid][0] = p; pr[tid][1] = q;
        if (applied && bcol == 0) atomicAdd(rot_count, 1);
      }
    }
    __syncthreads();
    const int u = tid / 16, col = bcol * 16 + (tid % 16);
    const int k = bp * EB + u;
    if (k >= half || col >= m) return;
    const int p = pr[u][0], q = pr[u][1];
    const double c = cs_r[u][0], s = cs_r[u][1];
    if (s == 0.0) return;
    const double wp = W[(int64_t)p * m + col], wq = W[(int64_t)q * m + col];
    W[(int64_t)p * m + col] = c * wp - s * wq;
    W[(int64_t)q * m + col] = s * wp + c * wq;
  }
}

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

// ---------------------------------------------------------------- launchers
hipError_t launch_eye(double* W, int m, hipStream_t st) {
  k_eye<<<(unsigned)(((int64_t)m * m + 255) / 256), 256, 0, st>>>(W, m);
  return hipGetLastError();
}
hipError_t launch_trace(const double* A, int m, double* out, hipStream_t st) {
  k_trace<<<1, 256, 0, st>>>(A, m, out);
  return hipGetLastError();
}
hipError_t launch_jacobi_round(const double* A, double* A2, double* W, int m, int t, double thr,
                               int* rot_count, hipStream_t st) {
  const int half = m / 2;
  const int gb = (half + EB - 1) / EB;
  const int nA = gb * gb;
  const int nW = gb * ((m + 15) / 16);
  k_jacobi_round<<<(unsigned)(nA + nW), 256, 0, st>>>(A, A2, W, m, t, thr, nA, rot_count);
  return hipGetLastError();
}
hipError_t launch_eig_sort(const double* A, const double* W, int m, int d, double* lam, double* Vt,
                           hipStream_t st) {
  k_eig_sort<<<(unsigned)d, 256, 0, st>>>(A, W, m, d, lam, Vt);
  return hipGetLastError();
}

}  // namespace adg
