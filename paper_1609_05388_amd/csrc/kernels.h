// Launchers of the gfx950 kernels (internal to the library).
#pragma once
#include "common.h"

namespace adg {

// k_prep.hip
// pmin/pmax (nchunks x m) and keep (m) may be null; with them keep[c] = 0
// marks a column holding one value only.
template <typename T>
hipError_t launch_mean(const T* A, int64_t n, int64_t m, int64_t ld, double* partial, int64_t nchunks,
                       int64_t rows_per_chunk, double* mu, int* nonfinite, hipStream_t st,
                       double* pmin = nullptr, double* pmax = nullptr, int* keep = nullptr);
hipError_t launch_compact_keep(const int* keep, int m, int* idx, int* k_out, hipStream_t st);
// FP64 centred copy of the columns colmap[0, m) (n x m); FP64 copy of the
// columns colmap[0, m) of an FP32 r x d matrix (r x m).
hipError_t launch_center64(const float* src, int64_t n, int64_t lds, const double* mu, const int* colmap, int64_t m,
                           double* dst, hipStream_t st);
hipError_t launch_cols64(const float* P, int64_t r, int64_t d, const int* colmap, int64_t m, double* dst,
                         hipStream_t st);
// colmap (m entries, may be null): source column of each destination column.
template <typename T>
hipError_t launch_center(const T* src, int64_t n, int64_t m, int64_t lds, const double* mu, float* dst,
                         int64_t ldd, int64_t n_pad, double* norm2, hipStream_t st, const int* colmap = nullptr);
hipError_t launch_row_terms(const double* norm2, double c_self, const double* norm2_other, double c_other,
                            int64_t n_pad, float2* terms, hipStream_t st);

// k_gemm64.hip
hipError_t launch_covariance(const float* X, int64_t n, int64_t d, const double* mu, double* part, int nsplit,
                             double* C, int64_t m_pad, hipStream_t st);
// C (m_pad x m_pad, zero padding) = the sum of nsplit d x d partial products
// in split order, element (i, j) taken from partial entry [min][max].
hipError_t launch_cov_reduce(const double* part, int nsplit, int64_t d, int64_t m_pad, double* C, hipStream_t st);
hipError_t launch_embed_f32(const float* X, int64_t n, int64_t d, const float* Pi, int64_t r, float* Y,
                            hipStream_t st);
hipError_t launch_proj_T(const double* S, int64_t k, int64_t d, const double* Vt, int64_t s, double* T,
                         hipStream_t st);
hipError_t launch_proj_SQ(const double* S, const double* T, int64_t k, int64_t s, const double* Vt, int64_t d,
                          float* Pi, double* Pi64, hipStream_t st);

// k_eig.hip
hipError_t launch_eye(double* W, int m, hipStream_t st);
hipError_t launch_trace(const double* A, int m, double* out, hipStream_t st);
hipError_t launch_eig_sort(const double* A, const double* W, int m, int d, double* lam, double* Vt,
                           hipStream_t st);
hipError_t launch_scatter_axes(const double* lam1, const double* Vt1, const int* idx, int d1, int d, double* lam,
                               double* Vt, hipStream_t st);

// k_dgemm.hip: FP64 MFMA products on 128 x 128 tiles (row-major operands).
// nt: C[m][n] = sum_k A[m][k] B[n][k];  nn: C[m][n] = sum_k A[m][k] B[k][n];
// tn: C[m][n] = sum_k A[k][m] B[k][n], split over k into nsplit partials
// C + s M ldc; syrk_upper: the upper 128 x 128 tiles of A^T A (A: K x M),
// split over k into nsplit partials part + s M M (row stride M).
hipError_t launch_dgemm_nt(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int64_t N,
                           int64_t K, double* C, int64_t ldc, hipStream_t st);
hipError_t launch_dgemm_nn(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int64_t N,
                           int64_t K, double* C, int64_t ldc, hipStream_t st);
hipError_t launch_dgemm_tn(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int64_t N,
                           int64_t K, int nsplit, double* C, int64_t ldc, hipStream_t st);
hipError_t launch_dgemm_syrk_upper(const double* A, int64_t lda, int64_t M, int64_t K, int nsplit, double* part,
                                   hipStream_t st);
int dgemm_tile();
// dst[i * ldd + c] = src[i * lds + c] for i < rows, c < cols (FP64).
hipError_t launch_copy_block64(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                               int64_t cols, hipStream_t st);
// *out = sum of a[e]^2 (FP64), through nparts block partials in part.
hipError_t launch_sumsq(const double* a, int64_t count, double* part, int nparts, double* out, hipStream_t st);

// k_ceiling.hip: a kernel of independent MFMAs only (kind 0 FP8 32x32x64,
// 1 BF16 32x32x16, 2 FP32 32x32x2) over mfma_ceiling_grid() workgroups of
// 256 threads; in: 1024 words, out: one float per thread, clk: the shader
// clock and 100 MHz counter deltas of workgroup 0.
int mfma_ceiling_grid();
hipError_t launch_mfma_ceiling(int kind, const int* in, float* out, unsigned long long* clk, int iters,
                               hipStream_t st);

// k_chol.hip: in-place Cholesky factor (lower, strict upper zeroed) of an
// SPD m x m column-major FP64 matrix, m <= chol_max_m(); *fail = 1 on a
// non-positive pivot.
hipError_t launch_cholesky(double* A, int m, int* fail, hipStream_t st);
int chol_max_m();

// k_eig_block.hip
// One round t of the block Jacobi method on the m x m matrix A (in place), W
// (= V^T, in place); Uall, Sall: per block pair JS x JS scratch; rotated: per
// block pair flag (nb / 2 ints); rot_count accumulates applied rotations.
hipError_t launch_bj_round(double* A, double* W, double* Uall, double* Sall, int* rotated, int m, int t,
                           double thr, int* rot_count, hipStream_t st);
int bj_block();

// k_proj.hip
hipError_t launch_jl_signs(uint64_t seed, int64_t k, int64_t d, double* S, hipStream_t st);
hipError_t launch_copy_rows(const double* Vt, int64_t rows, int64_t d, float* Pi, double* Pi64, hipStream_t st);

// k_pairs.hip
struct PairsView {
  const float* X; int ldx;      // centred points (n_pad x ldx)
  const float* Y; int ldy;      // centred images (n_pad x ldy)
  const float2* tx; const float2* ty;
  int n; int NT; int64_t ntiles;
};
// Early stop of a screen (MODE 0): pairs with q_lo > q_hi or q_hi < q_lo of
// these thresholds are certain to exceed the target distortion; the first 8
// go to pairs, *count (zeroed by the caller) counts them, and workgroups
// that start once *count is nonzero skip their tile (their records are left
// as they were).
struct ScreenStop {
  uint32_t* count; int2* pairs; float q_hi, q_lo;
};
// gcache: point-Gram cache (16384 floats per tile) or null; gmode 1 stores
// the tiles' point Grams there, 2 loads them instead of recomputing.  stop:
// null, or the early stop.
hipError_t launch_pairs_screen(const PairsView& v, TileRec* recs, float* gcache, int gmode, const ScreenStop* stop,
                               hipStream_t st);
// The point Gram of every tile into gcache (gmode 1 without images or tile
// records): the screens of a fit then load it (gmode 2).
hipError_t launch_pairs_gram_fill(const PairsView& v, float* gcache, hipStream_t st);
hipError_t launch_pairs_emit(const PairsView& v, const uint32_t* list, const CertDev* cd, int2* cand, uint32_t cap,
                             uint32_t* ncand, int grid, hipStream_t st);

// k_pairs_bf16.hip
struct PairsViewB {
  const __bf16* Xb; int ldx;    // hi/lo split points (n_pad rows of 2 * ldx bf16)
  const __bf16* Yb; int ldy;    // hi/lo split images
  const float2* tx; const float2* ty;
  int n; int NT; int64_t ntiles;
  const float* dscale = nullptr;   // scale of the compact D^2 cache (device), with gcache
};
hipError_t launch_split_bf16(const float* src, int64_t n_pad, int64_t m, int64_t lds, int64_t ldb, __bf16* dst,
                             hipStream_t st);
// The precision-form screens' cache is the compact D^2 cache: per tile the
// 16384 pairs' D2lo, rounded down to FP16 at a power-of-two scale (32 KB per
// tile; kDcacheBytesPerTile).  scale: one float on the device, from
// launch_dcache_scale over the points' row norms N_i (FP64, n_pad of them).
hipError_t launch_dcache_scale(const double* nx, int64_t n, float* scale, hipStream_t st);
// gcache: null, or the compact cache with gmode 2 (and v.dscale); gmode 1 is
// refused (the fill below writes the cache).
hipError_t launch_pairs_screen_bf16(const PairsViewB& v, TileRec* recs, float* gcache, int gmode,
                                    const ScreenStop* stop, hipStream_t st);
hipError_t launch_pairs_gram_fill_bf16(const PairsViewB& v, float* gcache, hipStream_t st);

// k_cert.hip
// part: nparts + 1 records of scratch.
hipError_t launch_seeds(const TileRec* recs, int64_t ntiles, TileRec* part, int nparts, int2* seeds, CertDev* cd,
                        hipStream_t st);
template <typename TY>
hipError_t launch_rescore(const float* X, int64_t d, const TY* Y, int64_t r, const int2* pairs,
                          const uint32_t* count_ptr, const int* count_i, uint32_t cap, PairVal* out, int grid,
                          hipStream_t st);
hipError_t launch_thresholds(const PairVal* seedv, CertDev* cd, hipStream_t st);
hipError_t launch_flag_tiles(const TileRec* recs, int64_t ntiles, CertDev* cd, uint32_t* list, hipStream_t st);
hipError_t launch_top2(const PairVal* vals, const uint32_t* count_ptr, uint32_t cap, PairVal* part, int nparts,
                       CertDev* cd, hipStream_t st);
// Appends the record pairs of the first min(*nsel, kmax) tiles of list to a
// witness pool (pool_n counts, slots past cap are dropped).
hipError_t launch_pool_gather(const TileRec* recs, const uint32_t* list, const uint32_t* nsel, uint32_t kmax,
                              int2* pool, uint32_t* pool_n, uint32_t cap, hipStream_t st);
// Witness pairs by direct differences: V (npairs x m) = x_i - x_j over the
// non-constant coordinates colmap[0..m) in FP64; then eq. (2) from V and its
// images W = V Pi^T (npairs x r).
hipError_t launch_pair_diffs(const float* X, int64_t d, const int* colmap, int64_t m, const int2* pairs,
                             int64_t npairs, double* V, hipStream_t st);
hipError_t launch_pair_ratio(const double* V, int64_t m, const double* W, int64_t r, const int2* pairs,
                             int64_t npairs, PairVal* out, hipStream_t st);
// cd->best = cd->second = no pair.
hipError_t launch_best_reset(CertDev* cd, hipStream_t st);

// k_gemm64.hip (general FP64 products of the randomized PCA)
hipError_t launch_gemm_nt(const double* A, int64_t M, int64_t K, int64_t lda, const double* B, int64_t N,
                          int64_t ldb, double* C, int64_t ldc, hipStream_t st);
hipError_t launch_gemm_nn(const double* A, int64_t M, int64_t K, int64_t lda, const double* B, int64_t N,
                          int64_t ldb, double* C, int64_t ldc, hipStream_t st);
// Q row i times lam_i^(-1/2), zero where lam_i <= rel lam_0 (lam decreasing).
hipError_t launch_scale_rows_isqrt(double* Q, int64_t rows, int64_t cols, const double* lam, double rel,
                                   hipStream_t st);

// k_gemm64.hip (sketch)
// G = Omega Xc (m x d, FP64) with Omega[a][i] = +-1/sqrt(m) from SplitMix64
// output (a << 32 | i) + 1 of seed `sseed`; split over points, partials summed.
hipError_t launch_sketch(const float* X, int64_t n, int64_t d, const double* mu, int m, uint64_t sseed, double* part,
                         int nsplit, double* G, hipStream_t st);
// K = G G^T (m x m, FP64) into an mp x mp zero-padded matrix.
hipError_t launch_gram_rows(const double* G, int m, int64_t d, double* K, int mp, hipStream_t st);
// Features from the sorted sketch eigenvalues lam (m values, decreasing).
hipError_t launch_sketch_features(const double* lam, int m, int64_t n, int64_t d, double eps, float* feat,
                                  hipStream_t st);

// k_eigvals.hip
// Eigenvalues (decreasing) of the symmetric m x m FP64 matrix A (row stride
// lda), m <= 128, by tridiagonal reduction and Sturm bisection in one
// workgroup.
hipError_t launch_sym_eigvals(const double* A, int m, int lda, double* lam, hipStream_t st);

// k_pairs_fp8.hip
// Per-row scaled OCP e4m3 copy of n_pad rows of m FP32 values (row stride
// lds): q (ldq bytes per row, zero padded), scale s_i, N_i = s_i^2 |q_i|^2.
hipError_t launch_quant_fp8(const float* src, int64_t n_pad, int64_t m, int64_t lds, int64_t ldq, unsigned char* q,
                            float* scale, double* norm2, hipStream_t st);
// sx null: unit point scales (the point side then comes from the fit's
// compact D^2 cache and these terms' point entries go unused).
hipError_t launch_fp8_terms(const double* nx, const double* ny, const float* sx, const float* sy, int64_t n_pad,
                            float4* t, hipStream_t st);
// Estimated q extremes per tile (ldx, ldy multiples of fp8_chunk()).  gcache:
// null, or the fit's compact D^2 cache (launch_pairs_gram_fill_bf16) with
// gmode 2 and its scale dscale; recs non-null.
hipError_t launch_pairs_screen_fp8(const unsigned char* Xq, int ldx, const unsigned char* Yq, int ldy,
                                   const float4* terms, int n, int NT, TileRec* recs, float* gcache, int gmode,
                                   const float* dscale, hipStream_t st);
// Indices of the >= K tiles with the largest estimated distortion appended to
// list (at most kmax unless a single tied bucket exceeds it; hist: scratch of
// kTopkHistWords words, cleared here; nsel zeroed, receives the count).
constexpr size_t kTopkHistWords = 514;
hipError_t launch_topk_tiles(const TileRec* recs, int64_t ntiles, uint32_t K, uint32_t kmax, uint32_t* hist,
                             uint32_t* thr, uint32_t* list, uint32_t* nsel, hipStream_t st);
int fp8_chunk();

// k_mlp.hip
struct MlpLayout {
  int in, in_pad, hidden;
  int64_t W1, b1, W2, b2, W3, b3, w4, b4, total;
};
struct MlpActs {
  float *A1, *A2, *A3, *dZ, *dZ2, *g;
  __bf16 *A1b, *A2b;
};
MlpLayout mlp_layout();
hipError_t mlp_forward(const MlpLayout& L, const float* p, const __bf16* pb, const __bf16* X, int B, MlpActs& a,
                       float* out, hipStream_t st);
hipError_t mlp_backward(const MlpLayout& L, const __bf16* pb, const __bf16* X, const float* y, int B, float tau,
                        MlpActs& a, const float* out, float* grad, float* loss, hipStream_t st);
hipError_t mlp_adam(float* p, __bf16* pb, const float* g, float* m, float* v, int64_t count, float lr, int step,
                    hipStream_t st);
hipError_t mlp_to_bf16(const float* src, __bf16* dst, int64_t count, hipStream_t st);

// k_knn.hip
struct KnnView {
  const float* Qp; const float* Dp;  // padded panels, row stride K
  int64_t K, m;                      // padded and true widths
  const float* nq32; const float* nd32;
  int64_t nq, nd;
  int QB, S, tps, NTd, excl;
};
hipError_t launch_knn_prep(const float* src, int64_t n, int64_t m, int64_t n_pad, int64_t K, float* dst,
                           double* n64, float* n32, int* nonfinite, hipStream_t st);
hipError_t launch_knn_max(const double* v, int64_t n, double* out, hipStream_t st);
hipError_t launch_knn_screen(const KnnView& v, uint64_t* keys, unsigned* tau_g, hipStream_t st);
hipError_t launch_knn_finish(const KnnView& v, const uint64_t* keys, const float* Q, const float* D,
                             const double* nq64, const double* ndmax, const unsigned* tau_g, double cK, double g64,
                             int k, int32_t* idx, double* dist, int* nfb, int* fb, hipStream_t st);
hipError_t launch_knn_fallback(const float* Q, const float* D, int64_t m, int64_t nd, int k, int excl, const int* fb,
                               int nfb, int32_t* idx, double* dist, hipStream_t st);
hipError_t launch_knn_vote(const int32_t* nn, int64_t nq, int k, const int32_t* label, int64_t nd, int n_labels,
                           int group, int32_t* out, int* bad, hipStream_t st);

}  // namespace adg
