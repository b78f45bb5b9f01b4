// Step a8: from the screen's tile records to the exact certificate.
//
//  1. reduce the tile records to the pair with the largest q upper bound and
//     the pair with the smallest q lower bound (the seeds);
//  2. re-evaluate the seeds exactly in FP64 by direct differences; their best
//     value L is a distortion actually attained, so the maximum is >= L;
//  3. thresholds: a pair can reach distortion L only if q_hi >= (1 + L)^2 or
//     q_lo <= (1 - L)^2; flag the tiles whose record reaches them;
//  4. (screen kernel, emit mode) list every pair of a flagged tile that reaches
//     them, and re-evaluate those exactly;
//  5. the largest exact value is the maximum of eq. (3): every pair left out
//     has an upper bound below L.
// Ties are broken towards the smallest (i, j).
#include "common.h"
#include "kernels.h"

namespace adg {

__device__ inline bool rec_hi_better(float v, int i, int j, float v2, int i2, int j2) {
  if (i2 < 0) return i >= 0;
  if (i < 0) return false;
  if (v != v2) return v > v2;
  return i != i2 ? i < i2 : j < j2;
}
__device__ inline bool rec_lo_better(float v, int i, int j, float v2, int i2, int j2) {
  if (i2 < 0) return i >= 0;
  if (i < 0) return false;
  if (v != v2) return v < v2;
  return i != i2 ? i < i2 : j < j2;
}

// Stage 1: each block reduces a strided slice of tiles to one record.
__global__ __launch_bounds__(256) void k_tiles_reduce(const TileRec* __restrict__ recs, int64_t ntiles,
                                                      TileRec* __restrict__ out) {
  __shared__ TileRec sh[256];
  TileRec b;
  b.qhi = -1.f; b.qlo = 3.0e38f; b.ihi = b.jhi = b.ilo = b.jlo = -1; b.pad0 = b.pad1 = 0;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < ntiles; t += (int64_t)gridDim.x * 256) {
    const TileRec r = recs[t];
    if (rec_hi_better(r.qhi, r.ihi, r.jhi, b.qhi, b.ihi, b.jhi)) { b.qhi = r.qhi; b.ihi = r.ihi; b.jhi = r.jhi; }
    if (rec_lo_better(r.qlo, r.ilo, r.jlo, b.qlo, b.ilo, b.jlo)) { b.qlo = r.qlo; b.ilo = r.ilo; b.jlo = r.jlo; }
  }
  sh[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      TileRec a = sh[threadIdx.x];
      const TileRec c = sh[threadIdx.x + o];
      if (rec_hi_better(c.qhi, c.ihi, c.jhi, a.qhi, a.ihi, a.jhi)) { a.qhi = c.qhi; a.ihi = c.ihi; a.jhi = c.jhi; }
      if (rec_lo_better(c.qlo, c.ilo, c.jlo, a.qlo, a.ilo, a.jlo)) { a.qlo = c.qlo; a.ilo = c.ilo; a.jlo = c.jlo; }
      sh[threadIdx.x] = a;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

// Stage 2: seeds[0] = best expansion pair, seeds[1] = best contraction pair
// (a missing seed repeats the other; n_seed counts valid ones).
__global__ void k_seeds(const TileRec* __restrict__ part, int nparts, int2* __restrict__ seeds,
                        CertDev* __restrict__ cd) {
  if (threadIdx.x != 0) return;
  TileRec b;
  b.qhi = -1.f; b.qlo = 3.0e38f; b.ihi = b.jhi = b.ilo = b.jlo = -1;
  for (int k = 0; k < nparts; ++k) {
    const TileRec r = part[k];
    if (rec_hi_better(r.qhi, r.ihi, r.jhi, b.qhi, b.ihi, b.jhi)) { b.qhi = r.qhi; b.ihi = r.ihi; b.jhi = r.jhi; }
    if (rec_lo_better(r.qlo, r.ilo, r.jlo, b.qlo, b.ilo, b.jlo)) { b.qlo = r.qlo; b.ilo = r.ilo; b.jlo = r.jlo; }
  }
  int ns = 0;
  if (b.ihi >= 0) seeds[ns++] = make_int2(b.ihi, b.jhi);
  if (b.ilo >= 0 && !(ns == 1 && b.ilo == b.ihi && b.jlo == b.jhi)) seeds[ns++] = make_int2(b.ilo, b.jlo);
  cd->n_seed = ns;
  cd->qhi_all = b.ihi >= 0 ? b.qhi : 0.0f;
  cd->qlo_all = b.ilo >= 0 ? b.qlo : 1.0f;
  cd->n_flagged = 0;
  cd->n_cand = 0;
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Exact FP64 distortion of listed pairs by direct differences, one wave per
// pair: D^2 = sum_l (x_il - x_jl)^2 over the original rows of X (FP32 values
// taken exactly), E^2 = sum_m (y_im - y_jm)^2 over the images (FP32 or FP64).
template <typename TY>
__global__ __launch_bounds__(256) void k_rescore(const float* __restrict__ X, int64_t d, const TY* __restrict__ Y,
                                                 int64_t r, const int2* __restrict__ pairs,
                                                 const uint32_t* __restrict__ count_ptr, const int* __restrict__ count_i,
                                                 uint32_t cap, PairVal* __restrict__ out) {
  uint32_t count = count_ptr ? *count_ptr : (uint32_t)*count_i;
  if (count > cap) count = cap;
  const int lane = threadIdx.x & 63;
  const uint32_t nw = gridDim.x * 4;
  for (uint32_t w = blockIdx.x * 4 + (threadIdx.x >> 6); w < count; w += nw) {
    const int2 pr = pairs[w];
    const float* xi = X + (int64_t)pr.x * d;
    const float* xj = X + (int64_t)pr.y * d;
    double D2 = 0.0, E2 = 0.0;
    for (int64_t l = lane; l < d; l += 64) {
      const double t = (double)xi[l] - (double)xj[l];
      D2 += t * t;
    }
    const TY* yi = Y + (int64_t)pr.x * r;
    const TY* yj = Y + (int64_t)pr.y * r;
    for (int64_t m = lane; m < r; m += 64) {
      const double t = (double)yi[m] - (double)yj[m];
      E2 += t * t;
    }
    D2 = wave_sum_d(D2);
    E2 = wave_sum_d(E2);
    if (lane == 0) {
      PairVal pv;
      pv.i = pr.x; pv.j = pr.y; pv.pad = 0;
      if (D2 == 0.0) { pv.v = -1.0; pv.side = 0; }
      else {
        const double ratio = sqrt(E2) / sqrt(D2);
        pv.v = fabs(ratio - 1.0);
        pv.side = ratio > 1.0 ? 1 : (ratio < 1.0 ? -1 : 0);
      }
      out[w] = pv;
    }
  }
}

__device__ inline float f32_dn(double x) {
  float f = (float)x;
  if ((double)f > x) f = nextafterf(f, -INFINITY);
  return f;
}
__device__ inline float f32_upr(double x) {
  float f = (float)x;
  if ((double)f < x) f = nextafterf(f, INFINITY);
  return f;
}

__device__ inline bool pv_better(const PairVal& a, const PairVal& b) {
  if (b.i < 0) return a.i >= 0;
  if (a.i < 0) return false;
  return pair_better(a.v, a.i, a.j, b.v, b.i, b.j);
}
__device__ inline void top2_insert(PairVal& b1, PairVal& b2, const PairVal& x) {
  if (x.i < 0 || x.v < 0.0) return;
  if (x.i == b1.i && x.j == b1.j) return;
  if (pv_better(x, b1)) { b2 = b1; b1 = x; return; }
  if (x.i == b2.i && x.j == b2.j) return;
  if (pv_better(x, b2)) b2 = x;
}
__device__ inline PairVal pv_none() {
  PairVal p;
  p.v = -1.0; p.i = -1; p.j = -1; p.side = 0; p.pad = 0;
  return p;
}

// Thresholds from the seeds' exact values: L = best seed distortion.
// thr_hi = (1 + L)^2 rounded down, thr_lo = (1 - L)^2 rounded up (L < 1).
__global__ void k_thresholds(const PairVal* __restrict__ seedv, CertDev* __restrict__ cd) {
  if (threadIdx.x != 0) return;
  PairVal b1 = pv_none(), b2 = pv_none();
  for (int k = 0; k < cd->n_seed; ++k) top2_insert(b1, b2, seedv[k]);
  cd->best = b1;
  cd->second = b2;
  const double L = b1.i >= 0 ? b1.v : 0.0;
  cd->bound_rest = L;
  cd->thr_hi = f32_dn((1.0 + L) * (1.0 + L));
  cd->thr_lo = L < 1.0 ? f32_upr((1.0 - L) * (1.0 - L)) : (L == 1.0 ? 0.0f : -1.0f);
}

__global__ __launch_bounds__(256) void k_flag_tiles(const TileRec* __restrict__ recs, int64_t ntiles,
                                                    CertDev* __restrict__ cd, uint32_t* __restrict__ list) {
  const float th = cd->thr_hi, tl = cd->thr_lo;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < ntiles; t += (int64_t)gridDim.x * 256) {
    const TileRec r = recs[t];
    if ((r.ihi >= 0 && r.qhi >= th) || (r.ilo >= 0 && r.qlo <= tl)) {
      const uint32_t pos = atomicAdd(&cd->n_flagged, 1u);
      list[pos] = (uint32_t)t;
    }
  }
}

// Top-2 over exact values (distinct pairs): stage 1 per block.
__global__ __launch_bounds__(256) void k_top2_partial(const PairVal* __restrict__ vals,
                                                      const uint32_t* __restrict__ count_ptr, uint32_t cap,
                                                      PairVal* __restrict__ part) {
  __shared__ PairVal s1[256], s2[256];
  uint32_t count = *count_ptr;
  if (count > cap) count = cap;
  PairVal b1 = pv_none(), b2 = pv_none();
  for (uint32_t k = blockIdx.x * 256 + threadIdx.x; k < count; k += gridDim.x * 256) top2_insert(b1, b2, vals[k]);
  s1[threadIdx.x] = b1;
  s2[threadIdx.x] = b2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      PairVal a1 = s1[threadIdx.x], a2 = s2[threadIdx.x];
      top2_insert(a1, a2, s1[threadIdx.x + o]);
      top2_insert(a1, a2, s2[threadIdx.x + o]);
      s1[threadIdx.x] = a1;
      s2[threadIdx.x] = a2;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1[0];
    part[2 * blockIdx.x + 1] = s2[0];
  }
}

// Stage 2: merge block partials into the certificate's best / runner-up.
__global__ void k_top2_final(const PairVal* __restrict__ part, int nparts, CertDev* __restrict__ cd) {
  if (threadIdx.x != 0) return;
  PairVal b1 = cd->best, b2 = cd->second;
  for (int k = 0; k < 2 * nparts; ++k) top2_insert(b1, b2, part[k]);
  cd->best = b1;
  cd->second = b2;
}

// Witness pool of a search: the record pairs (largest and smallest ratio
// bound) of selected tiles, appended at pool_n (slots past cap are dropped;
// pool_n keeps counting and readers clamp it to cap).
__global__ __launch_bounds__(256) void k_pool_gather(const TileRec* __restrict__ recs,
                                                     const uint32_t* __restrict__ list,
                                                     const uint32_t* __restrict__ nsel, uint32_t kmax,
                                                     int2* __restrict__ pool, uint32_t* __restrict__ pool_n,
                                                     uint32_t cap) {
  uint32_t m = *nsel;
  if (m > kmax) m = kmax;
  for (uint32_t t = blockIdx.x * 256 + threadIdx.x; t < m; t += gridDim.x * 256) {
    const TileRec r = recs[list[t]];
    if (r.ihi >= 0) {
      const uint32_t pos = atomicAdd(pool_n, 1u);
      if (pos < cap) pool[pos] = make_int2(r.ihi, r.jhi);
    }
    if (r.ilo >= 0 && !(r.ilo == r.ihi && r.jlo == r.jhi)) {
      const uint32_t pos = atomicAdd(pool_n, 1u);
      if (pos < cap) pool[pos] = make_int2(r.ilo, r.jlo);
    }
  }
}

// Witness pairs by direct differences (the oracle's definition of eq. (2)):
// V (npairs x m, row-major) = x_i - x_j in FP64 over the m non-constant
// coordinates colmap[0..m) (constant ones differ by exactly zero).
__global__ void k_pair_diffs(const float* __restrict__ X, int64_t d, const int* __restrict__ colmap, int64_t m,
                             const int2* __restrict__ pairs, int64_t npairs, double* __restrict__ V) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= npairs * m) return;
  const int64_t k = e / m;
  const int64_t col = colmap[e - k * m];
  const int2 pr = pairs[k];
  V[e] = (double)X[(int64_t)pr.x * d + col] - (double)X[(int64_t)pr.y * d + col];
}

// eq. (2) of each witness pair from its difference row v (length m) and its
// image row W = Pi v (length r), one wave per pair; same encoding as
// k_rescore.
__global__ __launch_bounds__(256) void k_pair_ratio(const double* __restrict__ V, int64_t m,
                                                    const double* __restrict__ W, int64_t r,
                                                    const int2* __restrict__ pairs, int64_t npairs,
                                                    PairVal* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= npairs) return;   // uniform per wave
  double D2 = 0.0, E2 = 0.0;
  for (int64_t l = lane; l < m; l += 64) {
    const double t = V[w * m + l];
    D2 += t * t;
  }
  for (int64_t l = lane; l < r; l += 64) {
    const double t = W[w * r + l];
    E2 += t * t;
  }
  D2 = wave_sum_d(D2);
  E2 = wave_sum_d(E2);
  if (lane == 0) {
    const int2 pr = pairs[w];
    PairVal pv;
    pv.i = pr.x; pv.j = pr.y; pv.pad = 0;
    if (D2 == 0.0) { pv.v = -1.0; pv.side = 0; }
    else {
      const double ratio = sqrt(E2) / sqrt(D2);
      pv.v = fabs(ratio - 1.0);
      pv.side = ratio > 1.0 ? 1 : (ratio < 1.0 ? -1 : 0);
    }
    out[w] = pv;
  }
}

__global__ void k_best_reset(CertDev* __restrict__ cd) {
  if (threadIdx.x != 0) return;
  cd->best = pv_none();
  cd->second = pv_none();
}

// ---------------------------------------------------------------- launchers
hipError_t launch_seeds(const TileRec* recs, int64_t ntiles, TileRec* part, int nparts, int2* seeds, CertDev* cd,
                        hipStream_t st) {
  // nparts block records, reduced again by one block into part[nparts]
  k_tiles_reduce<<<(unsigned)nparts, 256, 0, st>>>(recs, ntiles, part);
  k_tiles_reduce<<<1, 256, 0, st>>>(part, nparts, part + nparts);
  k_seeds<<<1, 64, 0, st>>>(part + nparts, 1, seeds, cd);
  return hipGetLastError();
}

template <typename TY>
hipError_t launch_rescore(const float* X, int64_t d, const TY* Y, int64_t r, const int2* pairs,
                          const uint32_t* count_ptr, const int* count_i, uint32_t cap, PairVal* out, int grid,
                          hipStream_t st) {
  k_rescore<TY><<<(unsigned)grid, 256, 0, st>>>(X, d, Y, r, pairs, count_ptr, count_i, cap, out);
  return hipGetLastError();
}
template hipError_t launch_rescore<float>(const float*, int64_t, const float*, int64_t, const int2*, const uint32_t*,
                                          const int*, uint32_t, PairVal*, int, hipStream_t);
template hipError_t launch_rescore<double>(const float*, int64_t, const double*, int64_t, const int2*, const uint32_t*,
                                           const int*, uint32_t, PairVal*, int, hipStream_t);

hipError_t launch_thresholds(const PairVal* seedv, CertDev* cd, hipStream_t st) {
  k_thresholds<<<1, 64, 0, st>>>(seedv, cd);
  return hipGetLastError();
}

hipError_t launch_flag_tiles(const TileRec* recs, int64_t ntiles, CertDev* cd, uint32_t* list, hipStream_t st) {
  int64_t g = (ntiles + 255) / 256;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  k_flag_tiles<<<(unsigned)g, 256, 0, st>>>(recs, ntiles, cd, list);
  return hipGetLastError();
}

hipError_t launch_top2(const PairVal* vals, const uint32_t* count_ptr, uint32_t cap, PairVal* part, int nparts,
                       CertDev* cd, hipStream_t st) {
  k_top2_partial<<<(unsigned)nparts, 256, 0, st>>>(vals, count_ptr, cap, part);
  k_top2_final<<<1, 64, 0, st>>>(part, nparts, cd);
  return hipGetLastError();
}

hipError_t launch_pool_gather(const TileRec* recs, const uint32_t* list, const uint32_t* nsel, uint32_t kmax,
                              int2* pool, uint32_t* pool_n, uint32_t cap, hipStream_t st) {
  k_pool_gather<<<(unsigned)((kmax + 255) / 256), 256, 0, st>>>(recs, list, nsel, kmax, pool, pool_n, cap);
  return hipGetLastError();
}

hipError_t launch_pair_diffs(const float* X, int64_t d, const int* colmap, int64_t m, const int2* pairs,
                             int64_t npairs, double* V, hipStream_t st) {
  if (npairs * m == 0) return hipSuccess;
  k_pair_diffs<<<(unsigned)((npairs * m + 255) / 256), 256, 0, st>>>(X, d, colmap, m, pairs, npairs, V);
  return hipGetLastError();
}

hipError_t launch_pair_ratio(const double* V, int64_t m, const double* W, int64_t r, const int2* pairs,
                             int64_t npairs, PairVal* out, hipStream_t st) {
  if (npairs == 0) return hipSuccess;
  k_pair_ratio<<<(unsigned)((npairs + 3) / 4), 256, 0, st>>>(V, m, W, r, pairs, npairs, out);
  return hipGetLastError();
}

hipError_t launch_best_reset(CertDev* cd, hipStream_t st) {
  k_best_reset<<<1, 64, 0, st>>>(cd);
  return hipGetLastError();
}

}  // namespace adg
