// FP64 MFMA GEMM of the fit's large products:
//   a2  covariance    C = Xc^T Xc           (n x d' centred rows; upper tiles, split over rows)
//   a6  embedding     Y = Xc Pi'^T          (n x r, once per probe)
//       Gram factor   M = Pi'^T Pi',  Z = Xc L
//       witnesses     W = V Pi'^T           (pool differences x map)
// One kernel on v_mfma_f64_16x16x4f64: 128 x 128 output tiles, four waves
// of 64 x 64 (4 x 4 MFMA tiles, 16 independent accumulators each), K in
// chunks of 16 staged through double-buffered LDS with the next chunk held
// in registers, so each chunk costs one barrier.  Both operands sit in LDS
// as [k][m] rows (m contiguous, padded so that a wave's fragment reads of
// four k rows fall into distinct bank halves).  Workgroups are renumbered so
// that consecutive tiles, which share an operand panel, run on one XCD and
// its L2.
#include "common.h"
#include "kernels.h"

namespace adg {

namespace {

constexpr int DT = 128;        // output tile (rows and columns)
constexpr int DK = 16;         // K chunk
constexpr int DLD = DT + 16;   // LDS row stride (doubles): rows k, k + 1 start 128 B apart mod 256 B
constexpr int kXcds = 8;

struct StoreD {   // C[split * split_stride + m * ldc + n]
  double* C; int64_t M, N, ldc, split_stride;
  __device__ void operator()(int64_t m, int64_t n, int split, double v) const {
    if (m < M && n < N) C[split * split_stride + m * ldc + n] = v;
  }
};

// Workgroup b of nwg, dispatched round-robin over the XCDs, as a logical
// index whose consecutive values share an XCD.
__device__ inline int64_t xcd_order(int64_t b, int64_t nwg) {
  const int64_t x = b % kXcds, i = b / kXcds;
  const int64_t q = nwg / kXcds, rem = nwg % kXcds;
  return x < rem ? x * (q + 1) + i : rem * (q + 1) + (x - rem) * q + i;
}

// Upper-triangle tile t (row-major over I <= J < NT) as (I, J).
__device__ inline void upper_tile(int64_t t, int64_t NT, int64_t& I, int64_t& J) {
  const double b = 2.0 * (double)NT + 1.0;
  int64_t i = (int64_t)((b - sqrt(b * b - 8.0 * (double)t)) * 0.5);
  if (i < 0) i = 0;
  if (i > NT - 1) i = NT - 1;
  while (i > 0 && i * NT - i * (i - 1) / 2 > t) --i;
  while (i + 1 < NT && (i + 1) * NT - (i + 1) * i / 2 <= t) ++i;
  I = i;
  J = i + (t - (i * NT - i * (i - 1) / 2));
}

// A DT x DK panel of an operand, eight consecutive doubles per thread
// (8-byte loads: 16-byte vector loads measured slower here).
// MN_CONTIG: element (mn, k) at p[k * ld + mn] (else p[mn * ld + k]).
template <bool MN_CONTIG>
struct Panel {
  double r[8];
  __device__ void load8(const double* src) {
#pragma unroll
    for (int u = 0; u < 8; ++u) r[u] = src[u];
  }
  __device__ void load(const double* __restrict__ p, int64_t ld, int64_t mn0, int64_t MN, int64_t k0, int64_t ke,
                       int tid) {
    if (MN_CONTIG) {
      const int kk = tid >> 4, mm = (tid & 15) * 8;
      const int64_t k = k0 + kk;
      const double* src = p + k * ld + mn0 + mm;
      if (k < ke && mn0 + mm + 8 <= MN) {
        load8(src);
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) r[u] = (k < ke && mn0 + mm + u < MN) ? src[u] : 0.0;
      }
    } else {
      const int mm = tid >> 1, kk = (tid & 1) * 8;
      const int64_t mn = mn0 + mm;
      const double* src = p + mn * ld + k0 + kk;
      if (mn < MN && k0 + kk + 8 <= ke) {
        load8(src);
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) r[u] = (mn < MN && k0 + kk + u < ke) ? src[u] : 0.0;
      }
    }
  }
  __device__ void stash(double (*S)[DLD], int tid) const {
    if (MN_CONTIG) {
      const int kk = tid >> 4, mm = (tid & 15) * 8;
#pragma unroll
      for (int u = 0; u < 8; ++u) S[kk][mm + u] = r[u];
    } else {
      const int mm = tid >> 1, kk = (tid & 1) * 8;
#pragma unroll
      for (int u = 0; u < 8; ++u) S[kk + u][mm] = r[u];
    }
  }
};

// C(m, n) = sum_k A(m, k) B(k, n) over the k of one split.
// AT: A(m, k) at A[k * lda + m] (else A[m * lda + k]).
// BT: B(k, n) at B[k * ldb + n] (else B[n * ldb + k]).
// TRI: the tiles are the upper triangle I <= J of tiles_m x tiles_m.
// The 1-D grid holds nsplit x ntiles workgroups.
template <bool AT, bool BT, bool TRI, class ST>
__global__ __launch_bounds__(256) void k_dgemm(const double* __restrict__ A, int64_t lda,
                                               const double* __restrict__ B, int64_t ldb, int64_t M, int64_t N,
                                               int64_t K, int64_t kps, int64_t tiles_n, int64_t ntiles, ST st) {
  __shared__ double As[2][DK][DLD];
  __shared__ double Bs[2][DK][DLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t logical = xcd_order(blockIdx.x, gridDim.x);
  const int split = (int)(logical / ntiles);
  const int64_t t = logical % ntiles;
  int64_t ti, tj;
  if (TRI) upper_tile(t, tiles_n, ti, tj);
  else { ti = t / tiles_n; tj = t % tiles_n; }
  const int64_t m0 = ti * DT, n0 = tj * DT;
  const int64_t kb = (int64_t)split * kps;
  const int64_t ke = kb + kps < K ? kb + kps : K;
  const int nch = ke > kb ? (int)((ke - kb + DK - 1) / DK) : 0;

  Panel<AT> pa;
  Panel<BT> pb;
  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (f64x4){0.0, 0.0, 0.0, 0.0};

  if (nch > 0) {
    pa.load(A, lda, m0, M, kb, ke, tid);
    pb.load(B, ldb, n0, N, kb, ke, tid);
    pa.stash(As[0], tid);
    pb.stash(Bs[0], tid);
    __syncthreads();
  }
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) {
      const int64_t k0 = kb + (int64_t)(c + 1) * DK;
      pa.load(A, lda, m0, M, k0, ke, tid);
      pb.load(B, ldb, n0, N, k0, ke, tid);
    }
#pragma unroll
    for (int ks = 0; ks < DK / 4; ++ks) {
      const int kr = ks * 4 + (lane >> 4);
      double fa[4], fb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) fa[i] = As[buf][kr][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) fb[j] = Bs[buf][kr][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    if (c + 1 < nch) {
      pa.stash(As[buf ^ 1], tid);
      pb.stash(Bs[buf ^ 1], tid);
    }
    __syncthreads();
  }
  // D layout of v_mfma_f64_16x16x4f64: lane l, register v -> (4 v + l / 16, l % 16).
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + wm * 64 + i * 16 + 4 * v + (lane >> 4);
        const int64_t n = n0 + wn * 64 + j * 16 + (lane & 15);
        st(m, n, split, acc[i][j][v]);
      }
}

template <bool AT, bool BT, bool TRI>
hipError_t run(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int64_t N, int64_t K,
               int nsplit, double* C, int64_t ldc, int64_t split_stride, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int64_t tm = (M + DT - 1) / DT, tn = (N + DT - 1) / DT;
  const int64_t ntiles = TRI ? tm * (tm + 1) / 2 : tm * tn;
  if (nsplit < 1) nsplit = 1;
  const int64_t kps = round_up((K + nsplit - 1) / nsplit, DK);
  const int64_t nwg = ntiles * nsplit;
  if (nwg >= ((int64_t)1 << 31) / 256) return hipErrorInvalidValue;
  StoreD s{C, M, N, ldc, split_stride};
  k_dgemm<AT, BT, TRI, StoreD><<<(unsigned)nwg, 256, 0, st>>>(A, lda, B, ldb, M, N, K, kps, TRI ? tm : tn, ntiles,
                                                               s);
  return hipGetLastError();
}

// out[e] = sum_b part[b][e], blocks in order.
__global__ void k_sumsq_part(const double* __restrict__ a, int64_t count, double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256)
    s += a[e] * a[e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
// dst[i * ldd + c] = src[i * lds + c] for rows i, columns c < cols.
__global__ __launch_bounds__(256) void k_copy_block64(const double* __restrict__ src, int64_t lds,
                                                      double* __restrict__ dst, int64_t ldd, int64_t rows,
                                                      int64_t cols) {
  for (int64_t i = blockIdx.x; i < rows; i += gridDim.x)
    for (int64_t c = threadIdx.x; c < cols; c += 256) dst[i * ldd + c] = src[i * lds + c];
}

__global__ void k_sum_parts(const double* __restrict__ part, int nparts, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += part[b];
  *out = s;
}

}  // namespace

hipError_t launch_dgemm_nt(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int64_t N,
                           int64_t K, double* C, int64_t ldc, hipStream_t st) {
  return run<false, false, false>(A, lda, B, ldb, M, N, K, 1, C, ldc, 0, st);
}

hipError_t launch_dgemm_nn(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int64_t N,
                           int64_t K, double* C, int64_t ldc, hipStream_t st) {
  return run<false, true, false>(A, lda, B, ldb, M, N, K, 1, C, ldc, 0, st);
}

hipError_t launch_dgemm_tn(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int64_t N,
                           int64_t K, int nsplit, double* C, int64_t ldc, hipStream_t st) {
  return run<true, true, false>(A, lda, B, ldb, M, N, K, nsplit, C, ldc, M * ldc, st);
}

hipError_t launch_dgemm_syrk_upper(const double* A, int64_t lda, int64_t M, int64_t K, int nsplit, double* part,
                                   hipStream_t st) {
  return run<true, true, true>(A, lda, A, lda, M, M, K, nsplit, part, M, M * M, st);
}

int dgemm_tile() { return DT; }

hipError_t launch_sumsq(const double* a, int64_t count, double* part, int nparts, double* out, hipStream_t st) {
  k_sumsq_part<<<nparts, 256, 0, st>>>(a, count, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_sum_parts<<<1, 64, 0, st>>>(part, nparts, out);
  return hipGetLastError();
}

hipError_t launch_copy_block64(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                               int64_t cols, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const int64_t g = rows < 8192 ? rows : 8192;
  k_copy_block64<<<(unsigned)g, 256, 0, st>>>(src, lds, dst, ldd, rows, cols);
  return hipGetLastError();
}

}  // namespace adg
