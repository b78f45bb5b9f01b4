// Step a3: block form of the parallel cyclic Jacobi method.
//
// The m x m FP64 matrix (m a multiple of 2 * JB, padding rows/columns zero)
// is cut into nb = m / JB index blocks.  A sweep has nb - 1 rounds; in each,
// the round-robin ordering pairs the blocks into nb / 2 disjoint pairs (P, Q).
// For each pair one workgroup rotates the 2 JB x 2 JB principal submatrix
// S = A[{P,Q}, {P,Q}] in LDS with the scalar two-sided Jacobi method,
// S <- U^T S U: in the first round of a sweep over every index pair of S (the
// pairs inside each block, once per sweep, and across), in the other rounds
// over the JB x JB pairs (p in P, q in Q) only, so a sweep rotates every index
// pair of the matrix about once, as one cyclic sweep of the scalar method in a
// parallel order.  Rotations with |S_pq| below the threshold are skipped.
// The round then applies the block-diagonal orthogonal J (the U's on their
// index sets): A <- J^T A J tile by tile (tile (PQ, RS) becomes
// U_PQ^T A_tile U_RS) and W <- J^T W, with W = V^T accumulating eigenvectors
// as rows.  A stays symmetric, so only its JB x JB blocks on and above the
// block diagonal are kept: a block (X, Y) with X > Y is read as the transpose
// of block (Y, X) and never written (the blocks below the diagonal of the
// input are left as they are), and one workgroup forms tile (PQ, RS) for pair
// indices ka <= kb only (half the A traffic and products of the full
// matrix).  Every tile and every W row block is read and written by one
// workgroup of the round, so both are updated in place; a subproblem that
// rotated nothing has U = I, and the products with it are skipped (a tile
// between two such pairs is left as it is), which makes the late sweeps,
// where most subproblems are already below the threshold, cheap.  The method
// has converged when a whole sweep skips every rotation.
#include "common.h"
#include "kernels.h"

namespace adg {

constexpr int JB = 32;        // index block
constexpr int JS = 2 * JB;    // subproblem size
constexpr int JLD = JS + 1;   // LDS row stride (doubles) of the subproblem
constexpr int SNT = 512;      // threads of a subproblem's workgroup: two waves per SIMD

// Pair k of round t of the round-robin ordering of `players` (even) players.
__device__ inline void rr_pair_b(int t, int k, int players, int& p, int& q) {
  const int M = players - 1;
  int a, b;
  if (k == 0) { a = 0; b = t % M + 1; }
  else { a = (t + k) % M + 1; b = ((t - k) % M + M) % M + 1; }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// Pair k of the round-robin ordering of JS players (the pairs rr_pair_b(r, k,
// JS) of inner rounds r = 0, 1, ...), advanced one round at a time: x and y
// hold (r + k) mod (JS - 1) and (r - k) mod (JS - 1), so a round costs two
// increments instead of two divisions.
struct RrStep {
  int x, y;
  bool first;   // k == 0: the pair (0, r mod (JS - 1) + 1)
  __device__ explicit RrStep(int k) : x(k % (JS - 1)), y((JS - 1 - k % (JS - 1)) % (JS - 1)), first(k == 0) {}
  __device__ void pair(int& p, int& q) const {
    const int a = first ? 0 : x + 1, b = first ? x + 1 : y + 1;
    p = a < b ? a : b;
    q = a < b ? b : a;
  }
  __device__ void next() {
    x = x + 1 == JS - 1 ? 0 : x + 1;
    y = y + 1 == JS - 1 ? 0 : y + 1;
  }
};

// Global index of local index i (0 <= i < JS) of block pair (P, Q).
__device__ inline int sub_index(int P, int Q, int i) { return i < JB ? P * JB + i : Q * JB + (i - JB); }

// Rotation (c, s) annihilating S[p][q] (Golub & Van Loan, sym.schur2: t = s / c
// is the root of t^2 + 2 tau t - 1 = 0 of smaller magnitude, tau = delta / a2,
// delta = S_qq - S_pp, a2 = 2 S_pq); (1, 0) when |S_pq| <= thr.  Without the
// divisions: with h = (delta^2 + a2^2)^(1/2) and w = |delta| + h,
// t = sgn(delta) a2 / w and 1 + t^2 = 2 h / w, so c = w / (2 h w)^(1/2) and
// s = t c = sgn(delta) a2 / (2 h w)^(1/2).  delta and a2 are first scaled by
// one power of two (exactly), which leaves c and s unchanged and keeps the
// squares in range.
__device__ inline void sub_rotation(const double* S, int p, int q, double thr, double& c, double& s) {
  const double apq = S[p * JLD + q];
  c = 1.0;
  s = 0.0;
  if (fabs(apq) > thr) {
    double dl = S[q * JLD + q] - S[p * JLD + p], a2 = 2.0 * apq;
    int e;
    (void)frexp(fmax(fabs(dl), fabs(a2)), &e);
    dl = ldexp(dl, -e);
    a2 = ldexp(a2, -e);
    const double h = sqrt(fma(dl, dl, a2 * a2));
    const double w = fabs(dl) + h;
    const double r = rsqrt(2.0 * h * w);
    c = w * r;
    s = (dl < 0.0 ? -a2 : a2) * r;
  }
}

// One workgroup per block pair (rr_pair_b(t, blockIdx.x)).  FULL: the
// round-robin over all 2 JB indices of S (2 JB - 1 inner rounds); else the
// cross pairs only, inner round r pairing p = i with q = JB + (i + r) mod JB
// (JB inner rounds).  Each inner round is one phase: a thread recomputes the
// rotations of the pairs it touches from the current S (every wave computes
// the JB rotations once: lanes l and l + 32 hold rotation l % 32, whose (c, s)
// the other lanes fetch by shuffles and whose index pair they recompute),
// writes its 2 x 2 blocks of J^T S J into the other LDS buffer and rotates its
// pair's columns of U; one barrier per inner round.  Writes U
// (JS x JS, U[i][j] = component i of vector j) and the final S; a subproblem
// with nothing above the threshold returns U = I without rotating.
template <bool FULL>
__global__ __launch_bounds__(SNT) void k_bj_solve(const double* __restrict__ A, int m, int nb, int t, double thr,
                                                  double* __restrict__ Uout, double* __restrict__ Sout,
                                                  int* __restrict__ rot_count, int* __restrict__ rotated) {
  extern __shared__ double lds_d[];
  double* const S0 = lds_d;
  double* const S1 = lds_d + JS * JLD;
  double* const U = lds_d + 2 * JS * JLD;
  __shared__ double off_sh[SNT / 64];
  __shared__ int applied_sh;
  const int pair = blockIdx.x;
  int P, Q;
  rr_pair_b(t, pair, nb, P, Q);
  const int tid = threadIdx.x;
  double off = 0.0;
  // all global reads first (in flight together), then the LDS writes; block
  // (Q, P), P < Q, is not read: it is the transpose of block (P, Q)
  double xv[JS * JS / SNT];
#pragma unroll
  for (int k = 0; k < JS * JS / SNT; ++k) {
    const int e = tid + SNT * k, i = e / JS, j = e % JS;
    xv[k] = (i >= JB && j < JB) ? 0.0 : A[(int64_t)sub_index(P, Q, i) * m + sub_index(P, Q, j)];
  }
#pragma unroll
  for (int k = 0; k < JS * JS / SNT; ++k) {
    const int e = tid + SNT * k, i = e / JS, j = e % JS;
    U[i * JLD + j] = (i == j) ? 1.0 : 0.0;
    if (i >= JB && j < JB) continue;
    const double x = xv[k];
    S0[i * JLD + j] = x;
    if (i < JB && j >= JB) S0[j * JLD + i] = x;
    if (FULL ? i != j : (i < JB && j >= JB)) off = fmax(off, fabs(x));
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) off = fmax(off, __shfl_xor(off, o, 64));
  if ((tid & 63) == 0) off_sh[tid >> 6] = off;
  if (tid == 0) applied_sh = 0;
  __syncthreads();
  off = off_sh[0];
#pragma unroll
  for (int w = 1; w < SNT / 64; ++w) off = fmax(off, off_sh[w]);
  int cur = 0;
  if (off > thr) {
    // thread -> column pair kb = tid % 32 and row pairs ka = tid / 32 + RS u
    // (u < JB / RS); the U update: pair kb, rows tid / 32 + RS v (v < JS / RS)
    constexpr int RS = SNT / JB;
    const int kb = tid & (JB - 1), ka0 = tid / JB;
    constexpr int rounds = FULL ? JS - 1 : JB;
    int nrot = 0;   // rotations applied by this lane's pair (lanes of wave 0 below JB)
    RrStep rb(kb), ra[JB / RS] = {RrStep(ka0), RrStep(ka0 + RS)};
    static_assert(JB / RS == 2, "two row pairs per thread");
    for (int r = 0; r < rounds; ++r) {
      const double* S = cur ? S1 : S0;
      double* S2 = cur ? S0 : S1;
      int pb, qb;
      if (FULL) { rb.pair(pb, qb); rb.next(); }
      else { pb = kb; qb = JB + ((kb + r) & (JB - 1)); }
      double cb, sbv;
      sub_rotation(S, pb, qb, thr, cb, sbv);
      nrot += (sbv != 0.0);
      // all LDS reads of the inner round first, then the arithmetic and the
      // writes, so that the reads' latencies overlap
      double ca[JB / RS], sa[JB / RS], mm[JB / RS][4];
      int pa[JB / RS], qa[JB / RS];
#pragma unroll
      for (int u = 0; u < JB / RS; ++u) {
        const int ka = ka0 + RS * u;
        ca[u] = __shfl(cb, ka, 64);
        sa[u] = __shfl(sbv, ka, 64);
        if (FULL) { ra[u].pair(pa[u], qa[u]); ra[u].next(); }
        else { pa[u] = ka; qa[u] = JB + ((ka + r) & (JB - 1)); }
        mm[u][0] = S[pa[u] * JLD + pb]; mm[u][1] = S[pa[u] * JLD + qb];
        mm[u][2] = S[qa[u] * JLD + pb]; mm[u][3] = S[qa[u] * JLD + qb];
      }
      double up[JS / RS], uq[JS / RS];
      if (sbv != 0.0) {
#pragma unroll
        for (int v = 0; v < JS / RS; ++v) {
          const int row = ka0 + RS * v;
          up[v] = U[row * JLD + pb];
          uq[v] = U[row * JLD + qb];
        }
      }
#pragma unroll
      for (int u = 0; u < JB / RS; ++u) {
        const int ka = ka0 + RS * u;
        const double m00 = mm[u][0], m01 = mm[u][1], m10 = mm[u][2], m11 = mm[u][3];
        const double r00 = ca[u] * m00 - sa[u] * m10, r01 = ca[u] * m01 - sa[u] * m11;
        const double r10 = sa[u] * m00 + ca[u] * m10, r11 = sa[u] * m01 + ca[u] * m11;
        double n00 = cb * r00 - sbv * r01, n01 = sbv * r00 + cb * r01;
        double n10 = cb * r10 - sbv * r11, n11 = sbv * r10 + cb * r11;
        if (ka == kb && sbv != 0.0) { n01 = 0.0; n10 = 0.0; }  // the annihilated pair
        S2[pa[u] * JLD + pb] = n00; S2[pa[u] * JLD + qb] = n01;
        S2[qa[u] * JLD + pb] = n10; S2[qa[u] * JLD + qb] = n11;
      }
      if (sbv != 0.0) {
#pragma unroll
        for (int v = 0; v < JS / RS; ++v) {
          const int row = ka0 + RS * v;
          U[row * JLD + pb] = cb * up[v] - sbv * uq[v];
          U[row * JLD + qb] = sbv * up[v] + cb * uq[v];
        }
      }
      __syncthreads();
      cur ^= 1;
    }
    if (tid < JB && nrot) atomicAdd(&applied_sh, nrot);
  }
  __syncthreads();
  const int applied = applied_sh;
  if (tid == 0) {
    rotated[pair] = applied ? 1 : 0;
    if (applied) atomicAdd(rot_count, applied);
  }
  if (!applied) return;   // U = I and S unchanged: nothing to write or apply
  const double* S = cur ? S1 : S0;
  double* Ug = Uout + (int64_t)pair * JS * JS;
  double* Sg = Sout + (int64_t)pair * JS * JS;
  for (int e = tid; e < JS * JS; e += SNT) {
    const int i = e / JS, j = e % JS;
    Ug[e] = U[i * JLD + j];
    Sg[e] = S[i * JLD + j];
  }
}

// One 32 x 32 quadrant (wave w: rows 32 (w / 2), columns 32 (w % 2)) of
// C = X^T Y for 64 x 64 matrices X (row stride LDX) and Y (row stride LDY),
// one in global memory (XG: X, else Y) and one in LDS: C[i][j] =
// sum_k X[k][i] Y[k][j], on v_mfma_f64_16x16x4f64 (A operand lane l: row
// l % 16, k = 4 ks + l / 16; B operand: column l % 16, same k; D register v:
// row 4 v + l / 16, column l % 16).  The global operand's values are all
// loaded before the products; the LDS operand's as they are needed.
template <int LDX, int LDY, bool XG>
__device__ inline void quad_xty(const double* __restrict__ X, const double* __restrict__ Y, f64x4 (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = (wave >> 1) * 32, c0 = (wave & 1) * 32;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (f64x4){0.0, 0.0, 0.0, 0.0};
  const double* G = XG ? X : Y;
  const int ldg = XG ? LDX : LDY, g0 = XG ? r0 : c0;
  double ga[JS / 4], gb[JS / 4];
#pragma unroll
  for (int ks = 0; ks < JS / 4; ++ks) {
    const int k = 4 * ks + (lane >> 4);
    ga[ks] = G[k * ldg + g0 + (lane & 15)];
    gb[ks] = G[k * ldg + g0 + 16 + (lane & 15)];
  }
#pragma unroll
  for (int ks = 0; ks < JS / 4; ++ks) {
    const int k = 4 * ks + (lane >> 4);
    double x0, x1, y0, y1;
    if (XG) {
      x0 = ga[ks]; x1 = gb[ks];
      y0 = Y[k * LDY + c0 + (lane & 15)]; y1 = Y[k * LDY + c0 + 16 + (lane & 15)];
    } else {
      x0 = X[k * LDX + r0 + (lane & 15)]; x1 = X[k * LDX + r0 + 16 + (lane & 15)];
      y0 = ga[ks]; y1 = gb[ks];
    }
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y1, acc[1][1], 0, 0, 0);
  }
}

// Tile (PQ, RS) of A (blocks P, Q of rows, R, S of columns, {P, Q} and {R, S}
// disjoint) into LDS, X[i][j] = A_tile[i][j] (X[j][i] when TR), from the blocks
// at or above the block diagonal: sub-block (xb, yb) is read from stored block
// (min, max) along its rows, so that the reads stay coalesced, and lands
// transposed when xb > yb.  All sixteen reads of a thread are in flight
// before the LDS writes.
template <bool TR>
__device__ inline void load_tile_upper(const double* __restrict__ A, int m, int P, int Q, int R, int S,
                                       double* X) {
  const int tid = threadIdx.x;
  constexpr int per = JB * JB / 256;
  double v[4 * per];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int xb = (b >> 1) ? Q : P, yb = (b & 1) ? S : R;
    const int rb = xb < yb ? xb : yb, cb = xb < yb ? yb : xb;
#pragma unroll
    for (int k = 0; k < per; ++k) {
      const int e = tid + 256 * k, hi = e / JB, lo = e % JB;
      v[b * per + k] = A[(int64_t)(rb * JB + hi) * m + cb * JB + lo];
    }
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int bi = b >> 1, bj = b & 1;
    const int xb = bi ? Q : P, yb = bj ? S : R;
    const bool above = xb < yb;
#pragma unroll
    for (int k = 0; k < per; ++k) {
      const int e = tid + 256 * k, hi = e / JB, lo = e % JB;
      const int li = bi * JB + (above ? hi : lo), lj = bj * JB + (above ? lo : hi);
      if (TR) X[lj * JLD + li] = v[b * per + k];
      else X[li * JLD + lj] = v[b * per + k];
    }
  }
}

// The new tile X[i][j] (LDS) into the blocks of A at or above the block
// diagonal: sub-block (xb, yb) goes to stored block (min, max), transposed
// when xb > yb.
__device__ inline void store_tile_upper(double* __restrict__ A, int m, int P, int Q, int R, int S,
                                        const double* X) {
  const int tid = threadIdx.x;
  constexpr int per = JB * JB / 256;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int bi = b >> 1, bj = b & 1;
    const int xb = bi ? Q : P, yb = bj ? S : R;
    const bool above = xb < yb;
    const int rb = above ? xb : yb, cb = above ? yb : xb;
#pragma unroll
    for (int k = 0; k < per; ++k) {
      const int e = tid + 256 * k, hi = e / JB, lo = e % JB;
      const int li = bi * JB + (above ? hi : lo), lj = bj * JB + (above ? lo : hi);
      A[(int64_t)(rb * JB + hi) * m + cb * JB + lo] = X[li * JLD + lj];
    }
  }
}

// Row ka and column kb (ka <= kb) of entry e of the upper triangle (with its
// diagonal) of an h x h array, stored row by row.
__device__ inline void tri_index(int e, int h, int& ka, int& kb) {
  const double b = 2.0 * h + 1.0;
  int a = (int)((b - sqrt(b * b - 8.0 * e)) * 0.5);
  // row a starts at a h - a (a - 1) / 2; correct the rounding of the root
  while (a > 0 && a * h - a * (a - 1) / 2 > e) --a;
  while ((a + 1) * h - (a + 1) * a / 2 <= e) ++a;
  ka = a;
  kb = a + (e - (a * h - a * (a - 1) / 2));
}

// Apply round t in place: A <- J^T A J (grid: (nb/2)(nb/2 + 1)/2 tiles of
// JS x JS, the block pairs ka <= kb) and W <- J^T W (grid: (nb/2) * (m / JS)
// tiles), one workgroup per tile: tile (PQ, RS) of A becomes
// U_PQ^T A_tile U_RS (two FP64 MFMA products with the intermediate kept
// transposed in LDS; one when either U is the identity, none when both are),
// a diagonal tile the solved S; only the blocks at or above the block diagonal
// are read and written.
__global__ __launch_bounds__(256) void k_bj_apply(double* __restrict__ A, double* __restrict__ W,
                                                  const double* __restrict__ Uall, const double* __restrict__ Sall,
                                                  const int* __restrict__ rotated, int m, int nb, int t) {
  // one 64 x 64 LDS buffer (the tile, then the intermediate); the rotations
  // U are read from global memory (L2 resident), so several workgroups share
  // a CU
  extern __shared__ double lds_d[];
  double* X = lds_d;
  const int half = nb / 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = (wave >> 1) * 32, c0w = (wave & 1) * 32;
  const int nA = half * (half + 1) / 2;
  f64x4 acc[2][2];
  if ((int)blockIdx.x < nA) {
    int ka, kb;
    tri_index((int)blockIdx.x, half, ka, kb);
    int P, Q, R, S;
    rr_pair_b(t, ka, nb, P, Q);
    rr_pair_b(t, kb, nb, R, S);
    const bool rot_a = rotated[ka] != 0, rot_b = rotated[kb] != 0;
    if (ka == kb) {  // diagonal tile: the solved subproblem itself
      if (!rot_a) return;
      const double* Sg = Sall + (int64_t)ka * JS * JS;
      double sv[JS * JS / 256];   // all reads in flight before the writes
#pragma unroll
      for (int k = 0; k < JS * JS / 256; ++k) sv[k] = Sg[tid + 256 * k];
#pragma unroll
      for (int k = 0; k < JS * JS / 256; ++k) {
        const int e = tid + 256 * k, i = e / JS, j = e % JS;
        if (i >= JB && j < JB) continue;   // block (Q, P), P < Q: not kept
        A[(int64_t)sub_index(P, Q, i) * m + sub_index(P, Q, j)] = sv[k];
      }
      return;
    }
    if (!rot_a && !rot_b) return;
    const double* ua = Uall + (int64_t)ka * JS * JS;
    const double* ub = Uall + (int64_t)kb * JS * JS;
    if (rot_a) {
      load_tile_upper<false>(A, m, P, Q, R, S, X);
      __syncthreads();
      quad_xty<JS, JLD, true>(ua, X, acc);    // T1 = Ua^T A_tile
      __syncthreads();
      if (rot_b) {
        // X <- T1^T (X[j][i] = T1[i][j])
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int i = r0 + a * 16 + 4 * v + (lane >> 4), j = c0w + b * 16 + (lane & 15);
              X[j * JLD + i] = acc[a][b][v];
            }
      }
    } else {
      // T1 = A_tile, held transposed: X[j][i] = A_tile[i][j]
      load_tile_upper<true>(A, m, P, Q, R, S, X);
    }
    if (rot_b) {
      __syncthreads();
      quad_xty<JLD, JS, false>(X, ub, acc);   // T1 Ub = (T1^T)^T Ub
    }
    __syncthreads();   // every wave is done reading X
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = r0 + a * 16 + 4 * v + (lane >> 4), j = c0w + b * 16 + (lane & 15);
          X[i * JLD + j] = acc[a][b][v];
        }
    __syncthreads();
    store_tile_upper(A, m, P, Q, R, S, X);
  } else {
    // W rows of pair ka, columns [c0, c0 + JS): W' = Ua^T W
    const int wb = blockIdx.x - nA;
    const int ncol = m / JS;
    const int ka = wb / ncol, c0 = (wb % ncol) * JS;
    if (rotated[ka] == 0) return;
    int P, Q;
    rr_pair_b(t, ka, nb, P, Q);
    const double* ua = Uall + (int64_t)ka * JS * JS;
    double wv[JS * JS / 256];   // all global reads in flight before the LDS writes
#pragma unroll
    for (int k = 0; k < JS * JS / 256; ++k) {
      const int e = tid + 256 * k, i = e / JS, j = e % JS;
      wv[k] = W[(int64_t)sub_index(P, Q, i) * m + c0 + j];
    }
#pragma unroll
    for (int k = 0; k < JS * JS / 256; ++k) {
      const int e = tid + 256 * k, i = e / JS, j = e % JS;
      X[i * JLD + j] = wv[k];
    }
    __syncthreads();
    quad_xty<JS, JLD, true>(ua, X, acc);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = r0 + a * 16 + 4 * v + (lane >> 4), j = c0w + b * 16 + (lane & 15);
          W[(int64_t)sub_index(P, Q, i) * m + c0 + j] = acc[a][b][v];
        }
  }
}

constexpr size_t kLdsSolve = 3 * JS * JLD * sizeof(double);
constexpr size_t kLdsApply = JS * JLD * sizeof(double);

hipError_t launch_bj_round(double* A, double* W, double* Uall, double* Sall, int* rotated, int m, int t,
                           double thr, int* rot_count, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bj_solve<true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsSolve);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bj_solve<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsSolve);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bj_apply), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kLdsApply);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int nb = m / JB;
  const int half = nb / 2;
  if (t == 0)
    k_bj_solve<true><<<(unsigned)half, SNT, kLdsSolve, st>>>(A, m, nb, t, thr, Uall, Sall, rot_count, rotated);
  else
    k_bj_solve<false><<<(unsigned)half, SNT, kLdsSolve, st>>>(A, m, nb, t, thr, Uall, Sall, rot_count, rotated);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_bj_apply<<<(unsigned)(half * (half + 1) / 2 + half * (m / JS)), 256, kLdsApply, st>>>(A, W, Uall, Sall, rotated,
                                                                                           m, nb, t);
  return hipGetLastError();
}

int bj_block() { return JB; }

}  // namespace adg
