/* adagio.h -- C ABI of the MI355X (gfx950) ADAGIO hot path.
 *
 * ADAGIO (Blasiok & Tsourakakis, arXiv 1609.05388) maps each point w of a
 * cloud T in R^d to (P w, S (w - P^T P w)), where P holds the top principal
 * directions of the centred cloud and S is a +-1/sqrt(k) Johnson-Lindenstrauss
 * matrix (Algorithm 1), and rates the map by its distortion: the largest,
 * over all pairs, of | ||f(x) - f(y)|| / ||x - y|| - 1 | (eqs. 2 and 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Arrays named X, Y, Pi, lambda, Vt are DEVICE pointers owned by the caller:
 *   contiguous, row-major, FP32 unless stated.  X is n x d (one point per
 *   row), Y is n x r, Pi is r x d.
 * - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *   All device work is ordered on it.  Entry points that return host scalars
 *   or check device results (fit, max_distortion, certify_map, pca,
 *   pca_randomized, project, knn, knn_vote) synchronise that stream before
 *   returning; embed and quantize_fp8 (no scratch) return without
 *   synchronising, and so do project_axes, project_family and the MLP calls
 *   when the workspace is kept (see below; later calls that share the kept
 *   workspace must then use the same stream).
 * - Sizes: 2 <= n <= 700000 points, 1 <= d <= 32768 coordinates, and n and d
 *   padded (to multiples of 128) with a product below 2^32; larger clouds
 *   return ADAGIO_E_UNSUPPORTED before any device work (a dispatch holds
 *   fewer than 2^32 work-items: the all-pairs screens launch one 256-thread
 *   workgroup per 128 x 128 tile slot, elementwise kernels one work-item per
 *   element of an n x d copy or a d x d matrix).
 * - Host structs (adagio_cert_t, adagio_opts_t, adagio_stats_t) are owned by
 *   the caller; opts may be NULL (defaults).
 * - Scratch memory: by default each call allocates the device workspace it
 *   needs (hipMalloc) and frees it before returning, after draining
 *   `stream` and the library's own streams; an entry point that uses
 *   scratch therefore returns with `stream` synchronised.  A caller that
 *   repeats calls can opt in to keeping one workspace per device across
 *   calls with adagio_keep_workspace(1); adagio_release() frees the current
 *   device's, and the library frees what is kept at process exit by itself
 *   (an exit handler registered after the HIP runtime has started, so it
 *   runs before the runtime's teardown).  A fit also makes two streams of
 *   its own on its device (one CU-masked), which every later call on that
 *   device reuses, kept or not, and which the same exit handler destroys.
 *   Calls are serialised by an internal lock.
 * - Return value: ADAGIO_OK (0) or a negative ADAGIO_E_* code.  On error the
 *   output buffers are unspecified and adagio_last_error() describes the
 *   failure (thread-local text).  Arguments are validated before any device
 *   work, so invalid arguments never touch the GPU.
 * - Results are deterministic: the same inputs, seed and device give bitwise
 *   identical outputs (timing fields aside; adagio_knn's n_fallback may also
 *   vary between runs, its answers do not; so may probe_delta of a fit probe
 *   whose screen stopped early, which is the first pair found, while the
 *   probe's outcome is fixed).
 */
#ifndef ADAGIO_H
#define ADAGIO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ADAGIO_OK 0
#define ADAGIO_E_INVALID_ARG (-1)   /* n < 2, d < 1, r outside [1, d], eps outside (0, 1), NULL pointer */
#define ADAGIO_E_NONFINITE (-2)     /* NaN or Inf in X (or Y) */
#define ADAGIO_E_HIP (-3)           /* HIP runtime error; adagio_last_error() has its text */
#define ADAGIO_E_OOM (-4)           /* device allocation failed */
#define ADAGIO_E_UNSUPPORTED (-5)   /* device is not gfx950, or size beyond the supported range */
#define ADAGIO_E_NO_CONVERGENCE (-6) /* eigensolver did not converge in its sweep limit */
#define ADAGIO_E_CAPACITY (-7)      /* more certificate candidates than the hard cap */
#define ADAGIO_E_NOT_CERTIFIED (-8) /* a certificate could not be completed */

/* Screening precision of the all-pairs certificate (the FP64 rescore and the
 * final value are exact in every mode). */
#define ADAGIO_SCREEN_F32 0      /* FP32 MFMA Gram, rigorous per-pair bounds   */
#define ADAGIO_SCREEN_BF16X3 1   /* BF16 hi/lo split, 3 BF16 MFMA products     */
#define ADAGIO_SCREEN_FP8 2      /* FP8 e4m3 per-row scaled screen: its 1024
                                    tiles of largest estimated distortion are
                                    re-screened with FP32 bounds and rescored;
                                    proves nothing about the other tiles
                                    (certified = 0, bound_rest = +inf); fits
                                    certify their result with BF16X3 */

/* Map family of a fit (Table 3 of Sec. 4.4 compares the three). */
#define ADAGIO_MAP_ADAGIO 0      /* Algorithm 1: [P ; S Q], floor(r/2) + ceil(r/2) rows */
#define ADAGIO_MAP_PCA 1         /* the top r principal directions alone          */
#define ADAGIO_MAP_JL 2          /* Lemma 1's r x d +-1/sqrt(r) matrix alone (no PCA) */

/* Principal directions of a fit. */
#define ADAGIO_PCA_EXACT 0       /* FP64 covariance + block Jacobi: every eigenpair */
#define ADAGIO_PCA_RANDOMIZED 1  /* Sec. 4.5's randomized PCA: top s + 10 directions
                                    by randomized subspace iteration              */

/* Target-dimension search. */
#define ADAGIO_SEARCH_BISECT 0   /* bisection over r in (0, d]                 */
#define ADAGIO_SEARCH_LEARNED 1  /* MLP prediction, certified, bisection fallback */

/* Result of an all-pairs certificate (eq. 3 over unordered pairs i < j). */
typedef struct adagio_cert {
    double max_distortion; /* exact (FP64) maximum of eq. (2); 0 when no valid pair */
    int64_t i, j;          /* argmax pair, i < j; smallest (i, j) among equal values; -1 if none */
    int32_t side;          /* +1 expansion (||f(x)-f(y)|| > ||x-y||), -1 contraction, 0 none */
    int32_t certified;     /* 1: every pair not re-evaluated in FP64 is proven <= max_distortion */
    double runner_up;      /* largest FP64 distortion among the other re-evaluated pairs (-1 if none) */
    int64_t i2, j2;        /* runner-up pair (-1 if none) */
    double bound_rest;     /* proven upper bound on the distortion of every pair not re-evaluated */
    int64_t n_rescored;    /* pairs re-evaluated exactly in FP64 */
    int64_t n_pairs;       /* pairs covered: n (n - 1) / 2 */
    int64_t n_flagged_tiles; /* pair tiles that needed a second, exact pass */
} adagio_cert_t;

/* Optional per-call timing and counters (filled when opts->stats != NULL). */
typedef struct adagio_stats {
    double t_total_ms;       /* host wall time of the call                        */
    double t_pca_ms;         /* centring + covariance + eigensolve (device events) */
    double t_search_ms;      /* the r search (device events)                      */
    double t_screen_ms;      /* sum of all-pairs screen kernel times              */
    double t_rescore_ms;     /* sum of candidate / rescore / emit stages          */
    int32_t n_certificates;  /* certificates computed                             */
    int32_t eig_sweeps;      /* Jacobi sweeps to convergence                      */
    int32_t n_fallback;      /* learned search: 1 when bisection was needed       */
    int32_t r_predicted;     /* learned search: the network's r (0 otherwise)     */
    int64_t n_flagged_tiles; /* summed over certificates                          */
    int64_t n_rescored;      /* summed over certificates                          */
    int32_t n_probes;        /* probes logged below, in call order (<= 48): the
                                certificates and, in a fit, the refuted probes    */
    int32_t n_screened;      /* how many of the certificates were FP8 screens     */
    int32_t probe_r[48];     /* target dimension of each probe                    */
    double probe_delta[48];  /* its exact max distortion (kinds 3 and 4 below: the
                                witness pair's exact distortion)                  */
    double probe_screen_ms[48]; /* its all-pairs screen kernel time (device events) */
    int32_t probe_gram[48];  /* its point Gram: 0 computed, 1 computed and stored in the
                                fit's point-Gram cache (no longer used by fits, which fill
                                the cache beforehand), 2 loaded from it (image Gram only),
                                3 none: the probe was refuted by a witness pair of the pool
                                (no screen; probe_delta is that pair's exact distortion, a
                                lower bound on the probe's maximum), 4 as 2 or 0, but the
                                screen stopped early at a pair certain to exceed eps
                                (probe_delta: that pair's exact distortion) */
    int32_t n_refuted;       /* fit: probes refuted by a witness pair (kinds 3 and 4, not
                                counted in n_certificates)                        */
    double t_gram_ms;        /* fit: the point-Gram cache fill (device events on the
                                library's second stream, overlapping the PCA); 0 when
                                the cache did not fit                             */
    int32_t probe_cols[48];  /* image columns its screen ran over: r, or d' (the non-constant
                                coordinates) when a map of r >= d' + 32 rows is screened
                                through the Gram factor; 0 for kind 3            */
} adagio_stats_t;

typedef struct adagio_opts {
    int32_t screen;          /* ADAGIO_SCREEN_*; default F32                      */
    int32_t search;          /* ADAGIO_SEARCH_*; default BISECT                   */
    int32_t max_candidates;  /* initial candidate capacity per certificate; 0 = default (2^20) */
    int32_t family;          /* ADAGIO_MAP_*; default ADAGIO (fit only)           */
    const float* predictor;  /* learned search: device pointer to the packed MLP parameters */
    adagio_stats_t* stats;   /* optional host output                              */
    int32_t pca;             /* ADAGIO_PCA_*; default EXACT (fit only)            */
    int32_t pca_iters;       /* randomized PCA: power iterations q (>= 0)         */
    int32_t no_witness;      /* fit: 1 = certify every probe in full (no refutation by
                                witness pairs, no early stop); default 0          */
    int32_t refine;          /* learned search: 1 = once the predicted r certifies,
                                probe downward (r / 1.25 each step while probes
                                pass), then bisect between the last failing and
                                the last passing r, so the result is
                                bisection-minimal like the plain search's (r - 1
                                fails); 2 = the same, but the bisection stops
                                once the last failing r is within 4% of the
                                last passing one (r - r_fail <= r / 25, so r is
                                within 1/0.96 of the smallest passing r when the
                                distortion falls with r); default 0 returns the
                                certified prediction                              */
} adagio_opts_t;

/* a1-a3.  Principal axes of the centred cloud (Sec. 2 PCA paragraph, eq. 4;
 * Sec. 3 first paragraph: P holds the top singular directions).
 * Computes mu = mean row (FP64), C = sum_i (x_i - mu)(x_i - mu)^T (FP64) and
 * its eigenpairs by a parallel cyclic Jacobi method.
 * Out: lambda (device, d doubles, decreasing), Vt (device, d x d doubles,
 * row i = unit eigenvector of lambda[i]).  Synchronises `stream`. */
int adagio_pca(const float* X, int64_t n, int64_t d, double* lambda, double* Vt, void* stream);

/* Randomized PCA, the paper's Adagio-Randomized-PCA variant (Sec. 4.1
 * "Implementation", Sec. 4.5; the randomized range finder of Halko,
 * Martinsson and Tropp): C = sum_i (x_i - mu)(x_i - mu)^T in FP64; a block of
 * ell sign vectors Omega (entry (a, l) from SplitMix64 output a * 2^32 + l + 1
 * of seed ^ 0x94D049BB133111EB, the same counter scheme as the JL signs);
 * Y = C Omega, then q more products Y = C Q, each time with Q an orthonormal
 * basis of the block (kept as rows; Lambda^-1/2 V^T Y^T from the eigenpairs
 * of the block's Gram, twice); finally the eigenpairs (W, lambda) of Q^T C Q
 * give the ell approximate principal directions (Q W)^T.  ell in [1, d],
 * power_iters = q >= 0.  Out: lambda (device, ell doubles, decreasing), Vt
 * (device, ell x d doubles, rows = unit directions).  Synchronises `stream`. */
int adagio_pca_randomized(const float* X, int64_t n, int64_t d, int32_t ell, int32_t power_iters, uint64_t seed,
                          double* lambda, double* Vt, void* stream);

/* a4-a5.  Algorithm 1's map at target dimension r from given principal axes:
 * s = floor(r/2) rows P = Vt[0:s], k = ceil(r/2) rows S Q = S - (S P^T) P with
 * S = B[0:k] / sqrt(k) (Lemma 1), the split of Sec. 4.1 "Implementation";
 * r = d returns Vt (no reduction).  B is the fixed +-1 matrix whose entry
 * (a, l) is the top bit of SplitMix64(seed) output number a * 2^32 + l + 1
 * (+1 when the bit is 0).  Vt: device d x d FP64 (rows = axes, decreasing
 * eigenvalue).  Pi_out: device r x d FP32.  Asynchronous. */
int adagio_project_axes(const double* Vt, int64_t d, int32_t r, uint64_t seed, float* Pi_out, void* stream);

/* f3.  The map of one family at a fixed r from the same sorted axes (the
 * rows compared in Table 3, Sec. 4.4): ADAGIO_MAP_ADAGIO is adagio_project_axes's map,
 * ADAGIO_MAP_PCA the top r rows of Vt, ADAGIO_MAP_JL the r x d +-1/sqrt(r)
 * sign matrix of Lemma 1 (the identity at r = d).  Vt: device d x d FP64;
 * Pi_out: device r x d FP32.  Asynchronous. */
int adagio_project_family(const double* Vt, int64_t d, int32_t r, int32_t family, uint64_t seed, float* Pi_out,
                          void* stream);

/* a1-a5.  Algorithm 1 at a fixed target dimension r (the fixed-r runs of
 * Sec. 4.2): PCA of X, then the map of adagio_project_axes.  Pi_out: device
 * r x d FP32.  Synchronises `stream`. */
int adagio_project(const float* X, int64_t n, int64_t d, int32_t r, uint64_t seed, float* Pi_out, void* stream);

/* a6.  The embedding f(w) = Pi w of every point (Algorithm 1's output line),
 * accumulated in FP64 and rounded once to FP32.  Y_out: device n x r FP32.
 * Asynchronous. */
int adagio_embed(const float* X, int64_t n, int64_t d, const float* Pi, int32_t r, float* Y_out, void* stream);

/* a7-a8.  Certificate of eq. (3) for a cloud X and its images Y (any map):
 * the exact maximum over unordered pairs i < j with x_i != x_j of eq. (2)
 * | ||y_i - y_j|| / ||x_i - x_j|| - 1 |.  An MFMA screen bounds every pair;
 * pairs whose bound reaches the best exact value are re-evaluated in FP64 by
 * direct differences of the given rows.  opts->screen picks the screen
 * precision; with ADAGIO_SCREEN_FP8 the result is the exact maximum over the
 * pairs of the screen's selected tiles only (a lower bound of eq. (3),
 * certified = 0).
 * cert_out: host.  Synchronises `stream`. */
int adagio_max_distortion(const float* X, int64_t n, int64_t d, const float* Y, int32_t r,
                          const adagio_opts_t* opts, adagio_cert_t* cert_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * certificate of adagio_max_distortion with the FP32 screen, every buffer
 * carved from one fixed 64 MiB device array that the library holds on each
 * GPU it runs on until the process ends; no hipMalloc, hipFree or allocating
 * library call.  The array holds the FP32 copies of the centred points and
 * images (about 4 n (d + r) bytes, n and d, r padded to 128 and 16), the
 * tile records and room for at least 65536 candidate pairs (32 bytes each);
 * inputs that need more return ADAGIO_E_UNSUPPORTED before any device work,
 * and so does opts->screen other than ADAGIO_SCREEN_F32.  The candidate
 * buffer does not grow: when the pairs to re-evaluate exceed the room left
 * (or opts->max_candidates), the result is an incomplete certificate
 * (certified = 0 with the proven bound_rest) where adagio_max_distortion
 * would grow its buffer and finish.  Every call on a GPU reuses that GPU's
 * array and leaves its contents behind (what must start at zero is cleared
 * by each call); calls are serialised by the library's lock and synchronise
 * `stream`, so two calls overlap only when made from separate processes,
 * which hold separate arrays.  cert_out: host.  Synchronises `stream`. */
int adagio_max_distortion_noalloc(const float* X, int64_t n, int64_t d, const float* Y, int32_t r,
                                  const adagio_opts_t* opts, adagio_cert_t* cert_out, void* stream);

/* a6-a8.  Certificate of eq. (3) for the linear map Pi (r x d FP32, device)
 * applied exactly: images are formed in FP64 from the FP32 entries of X and
 * Pi, so the result is the distortion of Pi itself.  When Pi has at least
 * d' + 32 rows (d' = coordinates of X that are not constant), the screen runs
 * over d' columns z = L^T x, L L^T = Pi'^T Pi' (the Cholesky factor of the
 * map's Gram over those coordinates), with the factor's rounding in its
 * bounds; the exact values are still taken from Pi x.  Synchronises
 * `stream`. */
int adagio_certify_map(const float* X, int64_t n, int64_t d, const float* Pi, int32_t r,
                       const adagio_opts_t* opts, adagio_cert_t* cert_out, void* stream);

/* a1-a9.  Fit: PCA once, then the smallest target dimension r whose map
 * (adagio_project_axes at r) has certified distortion <= eps, found by
 * bisection over r with lo = 0 and hi = d (Sec. 4.3's Fig. 6 and Sec. 4.4's Table 3 ask how many
 * dimensions a distortion level needs; the search procedure is this
 * library's).  eps is the absolute distortion target, in (0, 1).
 * Pi_out: device buffer of capacity d x d FP32; receives Pi (r x d).
 * r_out, s_out: host; cert_out: host, the certificate of the returned Pi.
 * opts->search = ADAGIO_SEARCH_LEARNED starts from the network's prediction
 * (opts->predictor) and falls back to bisection.  With ADAGIO_SCREEN_FP8 the
 * bisection decides on FP8 screens, then the result is certified with the
 * BF16 split screen; if that fails, certified bisection continues above it,
 * so the returned certificate is always a certificate.  The certificates of
 * the search share a point-Gram cache: the points do not change within a
 * fit, so each 128 x 128 tile's point side is kept in device memory and the
 * screens read it back and compute only the image Gram.  FP32 screens keep
 * the point Gram (64 KB per tile: 7.2 GB at n = 60000); the precision forms
 * keep, per pair, c / D2lo rounded up to FP16 (D2lo: the rigorous lower bound
 * on the squared distance that the screens' epilogue forms from the Gram;
 * c: a power of two from the largest row norm), 32 KB per tile.  The cache
 * is used when it fits in half of the free device memory, and the
 * certificate is the same either way.  The fit fills it with one launch on a
 * second stream of default priority: beside the PCA while the eigensolver
 * leaves the GPU mostly idle (padded covariance order up to 1024), after it
 * otherwise; `stream` waits for the fill before its first screen.  An FP8
 * fit fills the BF16 split cache, which its FP8 screens and its BF16 split
 * certificates both load.  opts->family = ADAGIO_MAP_PCA or ADAGIO_MAP_JL runs the same search
 * over the PCA-only or JL-only maps of Table 3 (at r = d: V^T, resp. the
 * identity); the learned search is for Algorithm 1's maps only.
 * opts->pca = ADAGIO_PCA_RANDOMIZED takes the principal directions from
 * adagio_pca_randomized with ell = s + 10 for the largest s the search has
 * needed so far (recomputed when a probe needs more; ell = d gives the exact
 * eigenbasis) and q = opts->pca_iters.
 * Refutation by witness pairs: a single pair whose exact eq. (2) value
 * exceeds eps shows that the maximum of eq. (3) exceeds eps, so a probe can
 * fail without an all-pairs screen.  After each certificate of a search, the
 * record pairs (the pair of largest and of smallest ratio bound) of its 256
 * tiles of largest bound join a pool of at most 16384 pairs; every later probe
 * first evaluates the pool in FP64 by direct differences Pi (x_i - x_j), before
 * it embeds the cloud, and fails when a pair exceeds eps + 1e-9 (a
 * margin far above the re-evaluation's rounding error, so that a refuted
 * probe is one its certificate would fail too).  A probe that the pool does
 * not refute runs its screen with an early stop: a pair whose rigorous bounds
 * put eq. (2) above eps + 2e-9 is recorded, workgroups that start after it
 * skip their tiles, and the pair re-evaluated above eps + 1e-9 fails the
 * probe (not while the first certificate fills the point-Gram cache).
 * Passing probes are certified in full as before, so r, Pi and the
 * certificate do not depend on either; opts->no_witness = 1 turns both off.
 * Synchronises `stream`. */
int adagio_fit(const float* X, int64_t n, int64_t d, double eps, uint64_t seed,
               const adagio_opts_t* opts, float* Pi_out, int32_t* r_out, int32_t* s_out,
               adagio_cert_t* cert_out, void* stream);

/* a10.  The FP8 screen's operand encoding: every row a_i of A (device, n x m
 * FP32, row-major) is scaled by s_i = max_l |a_il| / 448 (s_i = 1 for a zero
 * row) and rounded to nearest even into OCP FP8 e4m3 (bias 7, no infinities,
 * 448 the largest finite value): Q_out[i][l] = e4m3(a_il / s_i) (device, n x m
 * bytes), scale_out[i] = s_i (device, n floats), norm2_out[i] = s_i^2 |q_i|^2
 * accumulated in FP64 (device, n doubles).  Asynchronous. */
int adagio_quantize_fp8(const float* A, int64_t n, int64_t m, uint8_t* Q_out, float* scale_out, double* norm2_out,
                        void* stream);

/* a11.  Learned form (a method extension, not in the paper): the 80 input
 * features of the target-dimension predictor for cloud X and target eps.
 * G = Omega Xc is a JL sketch of the centred cloud with kSketchRows = 128 rows
 * of +-1/sqrt(128) signs (SplitMix64, seed ^ 0xD1B54A32D192ED03, counter
 * a * 2^32 + i + 1 for row a and point i); its eigenvalues lam_i = sigma_i^2
 * (decreasing) give f[i] = ln(sigma_i / ||sigma|| + 1e-6) / 4 for i < 64,
 * f[64] = ln(n) / 10, f[65] = ln(d) / 10, f[66] = 5 eps, f[67..79] = 0.
 * feat_out: device, 80 floats.  Synchronises `stream`. */
int adagio_sketch_features(const float* X, int64_t n, int64_t d, double eps, uint64_t seed, float* feat_out,
                           void* stream);

/* a11-a12.  Number of FP32 parameters of the predictor MLP: 67 inputs (padded
 * to 80) -> 256 -> 256 -> 256 (ReLU) -> 1, laid out as W1[256][80], b1[256],
 * W2[256][256], b2[256], W3[256][256], b3[256], w4[256], b4, 3 padding floats.
 * The output is the predicted ln(r / d). */
int64_t adagio_mlp_param_count(void);

/* a11.  Forward pass for B feature rows (device, B x 80 FP32) with FP32 master
 * parameters (device); products on BF16 MFMA with FP32 accumulation.  out:
 * device, B floats.  Asynchronous. */
int adagio_mlp_forward(const float* params, const float* feats, int32_t B, float* out, void* stream);

/* a12.  Pinball loss at level tau (0 < tau < 1) of targets - outputs, mean over
 * the batch, and its gradient w.r.t. all parameters (device, same layout as
 * params).  loss: device, 1 float.  Asynchronous. */
int adagio_mlp_grad(const float* params, const float* feats, const float* targets, int32_t B, float tau,
                    float* grad, float* loss, void* stream);

/* a12.  One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias corrected) on the
 * FP32 master params with the gradient of adagio_mlp_grad; adam_m, adam_v are
 * device state of the same layout (zero before step 1); step is 1-based.
 * loss: device, 1 float (loss before the step).  Asynchronous. */
int adagio_mlp_train_step(float* params, float* adam_m, float* adam_v, int32_t step, float lr, const float* feats,
                          const float* targets, int32_t B, float tau, float* loss, void* stream);

/* Timings and counts of one adagio_knn call. */
typedef struct adagio_knn_stats {
    double t_total_ms;       /* host wall time of the call                          */
    double t_prep_ms;        /* padded copies and row norms (device events)         */
    double t_screen_ms;      /* the FP32 MFMA screen (device events)                */
    double t_finish_ms;      /* candidate merge, FP64 rescoring, checks (events)    */
    double t_fallback_ms;    /* FP64 brute force of listed queries (events)         */
    int32_t splits;          /* database splits of the screen                       */
    int32_t n_fallback;      /* queries answered by the FP64 brute force            */
    int64_t reserved[4];
} adagio_knn_stats_t;

/* f4.  Exact k-nearest-neighbour queries, the operation of the
 * applications of Secs. 4.6 and 4.7: the 10-NN query of each descriptor of a query photo in the
 * image-retrieval experiment (Q = query descriptors, D = the database) and the
 * k = 30 nearest-neighbour graph of the classification experiment (Q = D,
 * exclude_self = 1), on original or embedded points.
 * Q: device nq x m FP32, D: device nd x m FP32, both dense row-major.  For
 * every query i the k database rows with the smallest squared distance
 * sum_l (q_l - x_l)^2, each difference, square and sum in FP64 in coordinate
 * order, equal distances ordered by the smaller row index; with
 * exclude_self = 1 query i skips database row i (nq <= nd).  1 <= k <= 32 and
 * k <= nd - exclude_self.  idx_out: device nq x k int32, dist_out: device
 * nq x k FP64, both ordered by (distance, index).  The answer is exact: an
 * FP32 MFMA screen keeps 32 candidates per query, and a query for which the
 * screen's error bound cannot prove that no other row enters the k best is
 * answered by FP64 brute force (stats_out->n_fallback counts them).
 * stats_out: host, may be NULL.  NaN or Inf inputs return ADAGIO_E_NONFINITE.
 * Synchronises `stream`. */
int adagio_knn(const float* Q, int64_t nq, const float* D, int64_t nd, int64_t m, int32_t k, int32_t exclude_self,
               int32_t* idx_out, double* dist_out, adagio_knn_stats_t* stats_out, void* stream);

/* f4.  Majority vote of the image-retrieval experiment (Sec. 4.6): queries come
 * in groups of `group` consecutive rows (one query photo; the last group may
 * be shorter); every neighbour in nn_idx (device nq x k int32, database row
 * indices) adds a vote to its label d_label[row] (device nd int32, in
 * [0, n_labels), n_labels <= 8192); label_out[g] (device, ceil(nq / group)
 * int32) is the label with most votes in group g, the smallest label among
 * ties (the paper draws at random among tied labels).  An index or label out
 * of range returns ADAGIO_E_INVALID_ARG.  Synchronises `stream`. */
int adagio_knn_vote(const int32_t* nn_idx, int64_t nq, int32_t k, const int32_t* d_label, int64_t nd,
                    int32_t n_labels, int32_t group, int32_t* label_out, void* stream);

/* Measurement aid for roofline figures (not a step of the method): the
 * matrix-core throughput of a kernel that issues nothing but independent
 * MFMAs of one kind on register operands (kind 0: FP8 e4m3 32x32x64, 1: BF16
 * 32x32x16, 2: FP32 32x32x2; four accumulators per wave, 1024 workgroups of
 * 256 threads), in TFLOP/s, and the shader clock in GHz that one workgroup
 * measured during it (s_memtime against the 100 MHz s_memrealtime).  The
 * published dense peaks assume the 2.4 GHz peak clock; under a sustained
 * MFMA load the clock settles lower.  tflops_out and ghz_out are host
 * doubles.  Allocates about 1 MB, runs four launches of ~2.5 ms (the last is
 * timed) and synchronises `stream`.  ADAGIO_E_INVALID_ARG for another kind. */
int adagio_mfma_ceiling(int32_t kind, double* tflops_out, double* ghz_out, void* stream);

/* Workspace ownership: keep = 1 keeps each device's workspace (buffers,
 * the fit's point-Gram cache, two streams and their events) across calls,
 * so that repeated calls skip allocation; keep = 0 (the default) frees every
 * call's workspace before it returns and frees what is kept now.  Any other
 * value returns ADAGIO_E_INVALID_ARG. */
int adagio_keep_workspace(int keep);

/* Frees the kept workspace of the current device (nothing when none is kept). */
int adagio_release(void);

/* Static text of a status code. */
const char* adagio_status_string(int status);

/* Thread-local description of the last error on this thread ("" if none). */
const char* adagio_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ADAGIO_H */
