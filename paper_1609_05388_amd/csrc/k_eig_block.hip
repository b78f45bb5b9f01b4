// Step a3: block form of the parallel cyclic Jacobi method.
//
// The m x m FP64 matrix (m a multiple of 2 * JB, padding rows/columns zero)
// is cut into nb = m / JB index blocks.  A sweep has nb - 1 rounds; in each,
// the round-robin ordering pairs the blocks into nb / 2 disjoint pairs (P, Q).
// For each pair one workgroup diagonalises the 2 JB x 2 JB principal
// submatrix S = A[{P,Q}, {P,Q}] to convergence with the scalar two-sided
// Jacobi method in LDS, S = U Lambda U^T (rotations below the threshold are
// skipped).  The round then applies the block-diagonal orthogonal J (the U's
// on their index sets): A <- J^T A J tile by tile (tile (PQ, RS) becomes
// U_PQ^T A_tile U_RS) and W <- J^T W, with W = V^T accumulating eigenvectors
// as rows.  The method has converged when a whole sweep skips every rotation.
#include "common.h"
#include "kernels.h"

namespace adg {

constexpr int JB = 32;        // index block
constexpr int JS = 2 * JB;    // subproblem size
constexpr int JLD = JS + 1;   // LDS row stride (doubles) of the subproblem

// Pair k of round t of the round-robin ordering of `players` (even) players.
__device__ inline void rr_pair_b(int t, int k, int players, int& p, int& q) {
  const int M = players - 1;
  int a, b;
  if (k == 0) { a = 0; b = t % M + 1; }
  else { a = (t + k) % M + 1; b = ((t - k) % M + M) % M + 1; }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// Global index of local index i (0 <= i < JS) of block pair (P, Q).
__device__ inline int sub_index(int P, int Q, int i) { return i < JB ? P * JB + i : Q * JB + (i - JB); }

// Rotation (c, s) annihilating S[p][q] (Golub & Van Loan, sym.schur2);
// (1, 0) when |S_pq| <= thr.
__device__ inline void sub_rotation(const double* S, int p, int q, double thr, double& c, double& s) {
  const double apq = S[p * JLD + q];
  c = 1.0;
  s = 0.0;
  if (fabs(apq) > thr) {
    const double app = S[p * JLD + p], aqq = S[q * JLD + q];
    const double tau = (aqq - app) / (2.0 * apq);
    const double tt = fabs(tau) > 1e150 ? 0.5 / tau : (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    c = 1.0 / sqrt(1.0 + tt * tt);
    s = tt * c;
  }
}

// One workgroup per block pair: `max_inner` sweeps of the scalar method on S
// (writes U, JS x JS row-major with U[i][j] = component i of vector j, and the
// final S).  Each inner round is one phase: a thread recomputes the rotations
// of the pairs it touches from the current S and writes its 2 x 2 blocks of
// J^T S J into the other LDS buffer, and rotates its pair's columns of U; one
// barrier per round.
__global__ __launch_bounds__(256) void k_bj_solve(const double* __restrict__ A, int m, int nb, int t, double thr,
                                                  int max_inner, double* __restrict__ Uout,
                                                  double* __restrict__ Sout, int* __restrict__ rot_count) {
  extern __shared__ double lds_d[];
  double* const S0 = lds_d;
  double* const S1 = lds_d + JS * JLD;
  double* const U = lds_d + 2 * JS * JLD;
  __shared__ int applied_sh;
  const int pair = blockIdx.x;
  int P, Q;
  rr_pair_b(t, pair, nb, P, Q);
  const int tid = threadIdx.x;
  for (int e = tid; e < JS * JS; e += 256) {
    const int i = e / JS, j = e % JS;
    S0[i * JLD + j] = A[(int64_t)sub_index(P, Q, i) * m + sub_index(P, Q, j)];
    U[i * JLD + j] = (i == j) ? 1.0 : 0.0;
  }
  if (tid == 0) applied_sh = 0;
  __syncthreads();
  int cur = 0;
  // thread -> column pair kb = tid % 32 and row pairs ka = tid / 32 + 8 u (u < 4);
  // the U update: pair kb, rows tid / 32 + 8 v (v < 8)
  const int kb = tid & 31, ka0 = tid >> 5;
  int total_applied = 0;
  for (int sw = 0; sw < max_inner; ++sw) {
    const int before = applied_sh;
    for (int r = 0; r < JS - 1; ++r) {
      const double* S = cur ? S1 : S0;
      double* S2 = cur ? S0 : S1;
      // every wave computes the 32 rotations of this round once (lane l and
      // lane l + 32 both hold rotation l % 32); threads fetch theirs by shuffle
      int pb, qb;
      rr_pair_b(r, kb, JS, pb, qb);
      double cb, sbv;
      sub_rotation(S, pb, qb, thr, cb, sbv);
      if (tid < 32 && sbv != 0.0) atomicAdd(&applied_sh, 1);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int ka = ka0 + 8 * u;
        const double ca = __shfl(cb, ka, 64), sa = __shfl(sbv, ka, 64);
        const int pa = __shfl(pb, ka, 64), qa = __shfl(qb, ka, 64);
        const double m00 = S[pa * JLD + pb], m01 = S[pa * JLD + qb];
        const double m10 = S[qa * JLD + pb], m11 = S[qa * JLD + qb];
        const double r00 = ca * m00 - sa * m10, r01 = ca * m01 - sa * m11;
        const double r10 = sa * m00 + ca * m10, r11 = sa * m01 + ca * m11;
        double n00 = cb * r00 - sbv * r01, n01 = sbv * r00 + cb * r01;
        double n10 = cb * r10 - sbv * r11, n11 = sbv * r10 + cb * r11;
        if (ka == kb && sbv != 0.0) { n01 = 0.0; n10 = 0.0; }  // the annihilated pair
        S2[pa * JLD + pb] = n00; S2[pa * JLD + qb] = n01;
        S2[qa * JLD + pb] = n10; S2[qa * JLD + qb] = n11;
      }
      if (sbv != 0.0) {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const int row = ka0 + 8 * v;
          const double up = U[row * JLD + pb], uq = U[row * JLD + qb];
          U[row * JLD + pb] = cb * up - sbv * uq;
          U[row * JLD + qb] = sbv * up + cb * uq;
        }
      }
      __syncthreads();
      cur ^= 1;
    }
    const int a = applied_sh - before;
    total_applied += a;
    if (a == 0) break;
  }
  const double* S = cur ? S1 : S0;
  double* Ug = Uout + (int64_t)pair * JS * JS;
  double* Sg = Sout + (int64_t)pair * JS * JS;
  for (int e = tid; e < JS * JS; e += 256) {
    const int i = e / JS, j = e % JS;
    Ug[e] = U[i * JLD + j];
    Sg[e] = S[i * JLD + j];
  }
  if (tid == 0 && total_applied) atomicAdd(rot_count, total_applied);
}

// Apply round t: A2 = J^T A J (grid: (nb/2)^2 tiles of JS x JS) and
// W <- J^T W (grid: (nb/2) * (m / JS) tiles), one workgroup per tile.
__global__ __launch_bounds__(256) void k_bj_apply(const double* __restrict__ A, double* __restrict__ A2,
                                                  double* __restrict__ W, const double* __restrict__ Uall,
                                                  const double* __restrict__ Sall, int m, int nb, int t) {
  extern __shared__ double lds_d[];
  double* T0 = lds_d;
  double* Ua = lds_d + JS * JLD;
  double* Ub = lds_d + 2 * JS * JLD;
  const int half = nb / 2;
  const int tid = threadIdx.x;
  const int nA = half * half;
  if ((int)blockIdx.x < nA) {
    const int ka = blockIdx.x / half, kb = blockIdx.x % half;
    int P, Q, R, S;
    rr_pair_b(t, ka, nb, P, Q);
    rr_pair_b(t, kb, nb, R, S);
    if (ka == kb) {  // diagonal tile: the solved subproblem itself
      const double* Sg = Sall + (int64_t)ka * JS * JS;
      for (int e = tid; e < JS * JS; e += 256) {
        const int i = e / JS, j = e % JS;
        A2[(int64_t)sub_index(P, Q, i) * m + sub_index(P, Q, j)] = Sg[e];
      }
      return;
    }
    const double* ua = Uall + (int64_t)ka * JS * JS;
    const double* ub = Uall + (int64_t)kb * JS * JS;
    for (int e = tid; e < JS * JS; e += 256) {
      const int i = e / JS, j = e % JS;
      T0[i * JLD + j] = A[(int64_t)sub_index(P, Q, i) * m + sub_index(R, S, j)];
      Ua[i * JLD + j] = ua[e];
      Ub[i * JLD + j] = ub[e];
    }
    __syncthreads();
    // T1 = Ua^T T0, kept in registers: thread owns 16 entries of column j
    const int j = tid % JS, i0 = (tid / JS) * 16;
    double t1[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) t1[u] = 0.0;
    for (int k = 0; k < JS; ++k) {
      const double x = T0[k * JLD + j];
#pragma unroll
      for (int u = 0; u < 16; ++u) t1[u] = fma(Ua[k * JLD + i0 + u], x, t1[u]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) T0[(i0 + u) * JLD + j] = t1[u];
    __syncthreads();
    // A2 tile = T1 Ub: thread owns 16 entries of row i
    const int i = tid % JS, j0 = (tid / JS) * 16;
    double o[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) o[u] = 0.0;
    for (int k = 0; k < JS; ++k) {
      const double x = T0[i * JLD + k];
#pragma unroll
      for (int u = 0; u < 16; ++u) o[u] = fma(x, Ub[k * JLD + j0 + u], o[u]);
    }
    const int64_t gi = sub_index(P, Q, i);
#pragma unroll
    for (int u = 0; u < 16; ++u) A2[gi * m + sub_index(R, S, j0 + u)] = o[u];
  } else {
    // W rows of pair ka, columns [c0, c0 + JS): W' = Ua^T W
    const int wb = blockIdx.x - nA;
    const int ncol = m / JS;
    const int ka = wb / ncol, c0 = (wb % ncol) * JS;
    int P, Q;
    rr_pair_b(t, ka, nb, P, Q);
    const double* ua = Uall + (int64_t)ka * JS * JS;
    for (int e = tid; e < JS * JS; e += 256) {
      const int i = e / JS, j = e % JS;
      T0[i * JLD + j] = W[(int64_t)sub_index(P, Q, i) * m + c0 + j];
      Ua[i * JLD + j] = ua[e];
    }
    __syncthreads();
    const int j = tid % JS, i0 = (tid / JS) * 16;
    double t1[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) t1[u] = 0.0;
    for (int k = 0; k < JS; ++k) {
      const double x = T0[k * JLD + j];
#pragma unroll
      for (int u = 0; u < 16; ++u) t1[u] = fma(Ua[k * JLD + i0 + u], x, t1[u]);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) W[(int64_t)sub_index(P, Q, i0 + u) * m + c0 + j] = t1[u];
  }
}

constexpr size_t kLdsSolve = 3 * JS * JLD * sizeof(double);
constexpr size_t kLdsApply = 3 * JS * JLD * sizeof(double);

hipError_t launch_bj_round(const double* A, double* A2, double* W, double* Uall, double* Sall, int m, int t,
                           double thr, int max_inner, int* rot_count, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bj_solve),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsSolve);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bj_apply), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kLdsApply);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int nb = m / JB;
  const int half = nb / 2;
  k_bj_solve<<<(unsigned)half, 256, kLdsSolve, st>>>(A, m, nb, t, thr, max_inner, Uall, Sall, rot_count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_bj_apply<<<(unsigned)(half * half + half * (m / JS)), 256, kLdsApply, st>>>(A, A2, W, Uall, Sall, m, nb, t);
  return hipGetLastError();
}

int bj_block() { return JB; }

}  // namespace adg
