// Host side of the C ABI declared in include/adagio.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/adagio.h"
#include "common.h"
#include "kernels.h"

namespace adg {

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

struct Fail {
  int code;
};

static void set_err(const char* fmt, const char* a = "", long long b = 0) {
  char buf[512];
  snprintf(buf, sizeof(buf), fmt, a, b);
  g_err = buf;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      set_err("%s (" #expr ", line %lld)", hipGetErrorString(e_), (long long)__LINE__); \
      throw Fail{e_ == hipErrorOutOfMemory ? ADAGIO_E_OOM : ADAGIO_E_HIP};            \
    }                                                                                 \
  } while (0)

#define ARGCHK(cond, msg)         \
  do {                            \
    if (!(cond)) {                \
      set_err("%s", msg);         \
      throw Fail{ADAGIO_E_INVALID_ARG}; \
    }                             \
  } while (0)

// --------------------------------------------------------------- workspace
// A device buffer that grows on demand and is freed with its owner (unless
// it was carved from a call's fixed arena).
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  bool owned = true;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p && owned) (void)hipFree(p);
  }
};

struct Workspace {
  DevBuf mu, colpart, nonfinite, Xc, nx, tx, covpart, A0, W, trace, rot, lam, Vt;
  DevBuf S, T, Pi, Pi64, Y64, Yc, ny, ty, muY;
  DevBuf recs, tparts, seeds, seedv, list, cand, vals, vparts, cd;
  DevBuf Xb, txb, Yb, tyb, bjU, bjS, bjRot;
  DevBuf Xq, sx, nxq, Yq, sy, nyq, q8terms, hist, kthr, gcache, dscale;
  DevBuf rpQ, rpY, rpG, rpV, rpLam;
  DevBuf skpart, skG, skK, sklam, skV, skfeat, mlp_pb, mlp_X, mlp_f, mlp_hb, mlp_grad, mlp_loss;
  DevBuf knQ, knD, knNq64, knNd64, knNq32, knNd32, knMax, knKeys, knFb, knCnt, knTau;
  DevBuf lam1, Vt1, colmap, colminmax, colkeep, xc64, pi64c, axy;
  DevBuf pool, pooln, wvals, wparts, wcd, wV, wW, stopn, stopp, gfM, gfFail, gfZ, nrm;
  // the device's library streams (borrowed from g_aux / g_aux2, never
  // destroyed here): aux runs the fit's point-Gram fill during its PCA
  hipStream_t aux = nullptr;
  hipStream_t aux2 = nullptr;  // non-blocking, all CUs: the fit's exact PCA beside the fill
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_t0 = nullptr, ev_t1 = nullptr, ev_pca = nullptr,
             ev_cov = nullptr;
  Workspace() = default;
  Workspace(const Workspace&) = delete;
  Workspace& operator=(const Workspace&) = delete;
  // Drains the library's streams (the device's, which it borrows: see
  // device_streams), then frees events and (member destructors) every
  // buffer.  Errors are ignored: this also runs while an error unwinds a call.
  ~Workspace() {
    for (hipStream_t q : {aux, aux2}) {
      if (q) (void)hipStreamSynchronize(q);
    }
    for (hipEvent_t e : {ev_in, ev_out, ev_t0, ev_t1, ev_pca, ev_cov}) {
      if (e) (void)hipEventDestroy(e);
    }
  }
};

// Calls are serialised by g_mu.  By default each call owns a workspace that
// it frees before returning.  With adagio_keep_workspace(1) every device
// keeps one workspace across calls (g_kept, heap objects that no static
// destructor touches); the library then registers, once, an exit handler
// that frees them: it is registered after the HIP runtime has initialised,
// so it runs before the runtime's own teardown.
static std::mutex g_mu;
static bool g_keep = false;
static Workspace* g_kept[64];
static bool g_checked[64];
static bool g_exit_hook = false;
// The library's two streams of each device (aux: CU-masked, aux2), made on a
// device's first fit and kept until the process ends, by workspaces kept
// across calls and by per-call ones alike: making and destroying a CU-masked
// stream costs ~20 ms (measured on MI355X), more than a small fit.
static hipStream_t g_aux[64], g_aux2[64];

static void release_kept_all() {
  int cur = -1;
  const bool have_cur = hipGetDevice(&cur) == hipSuccess;
  for (int dev = 0; dev < 64; ++dev) {
    if (!g_kept[dev]) continue;
    if (hipSetDevice(dev) == hipSuccess) delete g_kept[dev];
    g_kept[dev] = nullptr;
  }
  if (have_cur) (void)hipSetDevice(cur);
}

static void release_streams_all() {
  int cur = -1;
  const bool have_cur = hipGetDevice(&cur) == hipSuccess;
  for (int dev = 0; dev < 64; ++dev) {
    if (!g_aux[dev] && !g_aux2[dev]) continue;
    if (hipSetDevice(dev) == hipSuccess) {
      for (hipStream_t q : {g_aux[dev], g_aux2[dev]}) {
        if (q) {
          (void)hipStreamSynchronize(q);
          (void)hipStreamDestroy(q);
        }
      }
    }
    g_aux[dev] = g_aux2[dev] = nullptr;
  }
  if (have_cur) (void)hipSetDevice(cur);
}

static void release_at_exit() {
  // another thread may still be inside a call at exit: leave its memory to
  // the process teardown rather than free it under the call
  if (!g_mu.try_lock()) return;
  release_kept_all();
  release_streams_all();
  g_mu.unlock();
}

// A fixed device region that a call carves its buffers from instead of
// allocating (adagio_max_distortion_noalloc); set while such a call runs.
struct Arena {
  unsigned char* base = nullptr;
  size_t size = 0, used = 0;
};
static Arena* g_arena = nullptr;

template <typename T>
static T* ensure(DevBuf& b, size_t count) {
  size_t bytes = count * sizeof(T);
  if (bytes == 0) bytes = 256;
  if (b.cap < bytes) {
    if (g_arena) {
      // grows by carving a new piece (the old one stays unused)
      const size_t off = (size_t)round_up((int64_t)g_arena->used, 256);
      if (off > g_arena->size || bytes > g_arena->size - off) {
        set_err("scratch array exhausted%s (needs %lld more bytes)", "", (long long)(off + bytes - g_arena->size));
        throw Fail{ADAGIO_E_UNSUPPORTED};
      }
      if (b.p && b.owned) HIPCHK(hipFree(b.p));
      b.p = g_arena->base + off;
      b.cap = bytes;
      b.owned = false;
      g_arena->used = off + bytes;
      return static_cast<T*>(b.p);
    }
    if (b.p && b.owned) HIPCHK(hipFree(b.p));
    b.p = nullptr;
    b.cap = 0;
    b.owned = true;
    HIPCHK(hipMalloc(&b.p, bytes));
    b.cap = bytes;
  }
  return static_cast<T*>(b.p);
}

// The current device, checked to be gfx950 (once per device).
static int checked_device() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) {
    set_err("device index %s%lld out of range", "", dev);
    throw Fail{ADAGIO_E_UNSUPPORTED};
  }
  if (!g_checked[dev]) {
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
      set_err("device architecture %s is not gfx950%lld", prop.gcnArchName, 0);
      throw Fail{ADAGIO_E_UNSUPPORTED};
    }
    g_checked[dev] = true;
  }
  return dev;
}

// The workspace of one call on `st`: the device's kept workspace, or a fresh
// one that the call frees when it ends (after its stream has drained), on
// success and on error alike.
struct CallWs {
  hipStream_t st;
  Workspace* ws = nullptr;
  Workspace* own = nullptr;
  explicit CallWs(hipStream_t s) : st(s) {
    const int dev = checked_device();
    if (g_keep) {
      if (!g_kept[dev]) {
        g_kept[dev] = new Workspace();
        if (!g_exit_hook) g_exit_hook = atexit(release_at_exit) == 0;
      }
      ws = g_kept[dev];
      // work an earlier call left on the library's streams (a fit that ended
      // in an error) must not overlap this call's use of the workspace
      if (ws->aux) HIPCHK(hipStreamSynchronize(ws->aux));
      if (ws->aux2) HIPCHK(hipStreamSynchronize(ws->aux2));
    } else {
      own = new Workspace();
      ws = own;
    }
  }
  CallWs(const CallWs&) = delete;
  CallWs& operator=(const CallWs&) = delete;
  ~CallWs() {
    if (own) {
      (void)hipStreamSynchronize(st);
      delete own;
    }
  }
};

// --------------------------------------------------------------- timing
struct EvPair {
  hipEvent_t a = nullptr, b = nullptr;
  bool on = true;    // off: no events are created or recorded, ms() is 0
  void begin(hipStream_t st) {
    if (!on) return;
    if (!a) { HIPCHK(hipEventCreate(&a)); HIPCHK(hipEventCreate(&b)); }
    HIPCHK(hipEventRecord(a, st));
  }
  void end(hipStream_t st) {
    if (on) HIPCHK(hipEventRecord(b, st));
  }
  double ms() {
    if (!on) return 0.0;
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, a, b));
    return (double)t;
  }
  ~EvPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// ------------------------------------------------------------ point state
// Centred FP32 points and their bound terms, shared by every certificate of
// one call.
struct Points {
  const float* X = nullptr;
  int64_t n = 0, d = 0, n_pad = 0, ldx = 0;
  int64_t dx = 0;            // columns of the screens' copies (non-constant columns of X)
  const int* colmap = nullptr;  // those columns, ascending (device)
  mutable double* xc64 = nullptr;  // FP64 centred copy of those columns (n x dx), on first use
  double* mu = nullptr;
  float* Xc = nullptr;
  double* nx = nullptr;
  float2* tx = nullptr;
  int screen = ADAGIO_SCREEN_F32;
  int64_t ldxb = 0;          // BF16 split (screen = BF16X3 or FP8)
  __bf16* Xb = nullptr;
  float2* txb = nullptr;
  int64_t ldxq = 0;          // per-row scaled e4m3 copy (screen = FP8)
  unsigned char* Xq = nullptr;
  float* sx = nullptr;
  double* nxq = nullptr;
  // FP8 screens of a fit load the BF16 split point Gram from the fit's cache
  // (unscaled, of the centred rows): their row terms take N = ||a||^2 and unit
  // point scales
  bool xgram_split = false;
  // scale of the fit's compact D^2 cache (precision-form fits with a cache)
  float* dscale = nullptr;
};

// Column means (FP64) of the n x m rows of A.  With colmap, also the columns
// that hold more than one value: colmap[0, k) lists them ascending and k is
// returned (m without colmap); the others have exactly zero centred entries.
static int64_t mean_rows(Workspace& ws, const float* A, int64_t n, int64_t m, int64_t ld, double* mu, hipStream_t st,
                         int* colmap = nullptr) {
  const int64_t rows_per_chunk = 512;
  const int64_t nch = (n + rows_per_chunk - 1) / rows_per_chunk;
  double* part = ensure<double>(ws.colpart, (size_t)(nch * m));
  int* flag = ensure<int>(ws.nonfinite, 2);   // [0] non-finite, [1] kept columns
  HIPCHK(hipMemsetAsync(flag, 0, 2 * sizeof(int), st));
  if (colmap) {
    double* pmm = ensure<double>(ws.colminmax, (size_t)(2 * nch * m));
    int* keep = ensure<int>(ws.colkeep, (size_t)m);
    HIPCHK(launch_mean<float>(A, n, m, ld, part, nch, rows_per_chunk, mu, flag, st, pmm, pmm + nch * m, keep));
    HIPCHK(launch_compact_keep(keep, (int)m, colmap, flag + 1, st));
  } else {
    HIPCHK(launch_mean<float>(A, n, m, ld, part, nch, rows_per_chunk, mu, flag, st));
  }
  int h[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(h, flag, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (h[0]) {
    set_err("input contains NaN or Inf%s%lld", "", 0);
    throw Fail{ADAGIO_E_NONFINITE};
  }
  return colmap ? (int64_t)h[1] : m;
}

// Bound constant for an FP32 Gram screen over K (padded) terms: covers the
// rounding of centring, of the row norms, of the MFMA dot product (gamma_K),
// of the epilogue's add and fma, and an 8u margin for the reciprocal.
static double screen_const(int64_t K) { return ((double)K + 32.0) * kU32 * 1.001; }

// The same for the BF16 split Gram (x = hi + lo + e, three BF16 products):
// dropped terms 3.01 * 2^-16 (= 770.6 u) and FP32 accumulation of 3K
// products of total size 1.012 sum |x||y| (3.04 K u), in place of gamma_K.
static double screen_const_bf16(int64_t K) { return (3.05 * (double)K + 771.0 + 32.0) * kU32 * 1.001; }
static const int64_t kChunkBf16 = 32;
static Points prep_points(Workspace& ws, const float* X, int64_t n, int64_t d, hipStream_t st,
                          int screen = ADAGIO_SCREEN_F32) {
  Points p;
  p.screen = screen;
  p.X = X;
  p.n = n;
  p.d = d;
  p.n_pad = round_up(n, kTile);
  p.mu = ensure<double>(ws.mu, (size_t)d);
  // Columns that hold one value only centre to exact zeros and add nothing
  // to any distance or Gram entry: the screens' copies leave them out.
  int* colmap = ensure<int>(ws.colmap, (size_t)d);
  p.dx = mean_rows(ws, X, n, d, d, p.mu, st, colmap);
  p.colmap = colmap;
  const int64_t dxc = std::max<int64_t>(p.dx, 1);
  p.ldx = round_up(dxc, kChunk);
  p.Xc = ensure<float>(ws.Xc, (size_t)(p.n_pad * p.ldx));
  p.nx = ensure<double>(ws.nx, (size_t)p.n_pad);
  p.tx = ensure<float2>(ws.tx, (size_t)p.n_pad);
  HIPCHK(launch_center<float>(X, n, p.dx, d, p.mu, p.Xc, p.ldx, p.n_pad, p.nx, st, colmap));
  HIPCHK(launch_row_terms(p.nx, screen_const(p.ldx), nullptr, 0.0, p.n_pad, p.tx, st));
  // The FP8 screen ranks pairs only; its fits end with a BF16 split
  // certificate, so both copies are made.
  if (screen == ADAGIO_SCREEN_BF16X3 || screen == ADAGIO_SCREEN_FP8) {
    p.ldxb = round_up(dxc, kChunkBf16);
    p.Xb = ensure<__bf16>(ws.Xb, (size_t)(p.n_pad * 2 * p.ldxb));
    p.txb = ensure<float2>(ws.txb, (size_t)p.n_pad);
    HIPCHK(launch_split_bf16(p.Xc, p.n_pad, p.dx, p.ldx, p.ldxb, p.Xb, st));
    HIPCHK(launch_row_terms(p.nx, screen_const_bf16(p.ldxb), nullptr, 0.0, p.n_pad, p.txb, st));
  }
  if (screen == ADAGIO_SCREEN_FP8) {
    p.ldxq = round_up(dxc, fp8_chunk());
    p.Xq = ensure<unsigned char>(ws.Xq, (size_t)(p.n_pad * p.ldxq));
    p.sx = ensure<float>(ws.sx, (size_t)p.n_pad);
    p.nxq = ensure<double>(ws.nxq, (size_t)p.n_pad);
    HIPCHK(launch_quant_fp8(p.Xc, p.n_pad, p.dx, p.ldx, p.ldxq, p.Xq, p.sx, p.nxq, st));
  }
  return p;
}

// ---------------------------------------------------------------- PCA
struct Axes {
  double* lam = nullptr;
  double* Vt = nullptr;  // d x d, rows = eigenvectors, decreasing eigenvalue
  int sweeps = 0;
};

// Eigenpairs of the symmetric m x m FP64 matrix in A (m a multiple of two
// Jacobi blocks, zero outside the leading d x d); only its Jacobi blocks on
// and above the block diagonal are read, and they are overwritten (the
// others are left stale).  Writes lam (d, decreasing) and Vt (d x d, rows =
// eigenvectors); returns sweeps.
static int jacobi_eig(Workspace& ws, double* A, int m, int64_t d, double* lam, double* Vt, hipStream_t st) {
  const int JB = bj_block();
  const int nb = m / JB;
  double* W = ensure<double>(ws.W, (size_t)m * m);
  double* Ub = ensure<double>(ws.bjU, (size_t)(nb / 2) * 4 * JB * JB);
  double* Sb = ensure<double>(ws.bjS, (size_t)(nb / 2) * 4 * JB * JB);
  int* rotated = ensure<int>(ws.bjRot, (size_t)(nb / 2));
  HIPCHK(launch_eye(W, m, st));
  double* tr = ensure<double>(ws.trace, 1);
  HIPCHK(launch_trace(A, m, tr, st));
  double trace = 0.0;
  HIPCHK(hipMemcpyAsync(&trace, tr, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // Rotations whose off-diagonal entry is at most 4 u64 trace(A) are skipped
  // (trace >= ||A||_F for PSD A; this sits above the rounding floor of the
  // tile products); the method has converged when a whole sweep skips every
  // rotation.
  const double thr = 4.0 * kU64 * trace;
  int* rot = ensure<int>(ws.rot, 1);
  const int max_sweeps = 40;
  int sweep = 0;
  bool converged = false;
  for (; sweep < max_sweeps && !converged; ++sweep) {
    HIPCHK(hipMemsetAsync(rot, 0, sizeof(int), st));
    for (int t = 0; t < nb - 1; ++t) HIPCHK(launch_bj_round(A, W, Ub, Sb, rotated, m, t, thr, rot, st));
    int h = 0;
    HIPCHK(hipMemcpyAsync(&h, rot, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    converged = (h == 0);
  }
  if (!converged) {
    set_err("Jacobi eigensolver did not converge in %s%lld sweeps", "", max_sweeps);
    throw Fail{ADAGIO_E_NO_CONVERGENCE};
  }
  HIPCHK(launch_eig_sort(A, W, m, (int)d, lam, Vt, st));
  return sweep;
}

// C = sum_i (x_i - mu)(x_i - mu)^T over all d coordinates into ws.A0 (m x m,
// zero padding; m = d rounded up to a multiple of two Jacobi blocks), by the
// library's own FP64 MFMA kernel (the randomized PCA's input).
static double* covariance(Workspace& ws, const Points& p, int m, hipStream_t st) {
  const int64_t d = p.d;
  // split-K over points so that the grid fills the GPU
  const int64_t NT = (d + 63) / 64;
  const int64_t ntiles = NT * (NT + 1) / 2;
  int nsplit = (int)((2048 + ntiles - 1) / ntiles);
  const int64_t max_split = (p.n + 255) / 256;
  if (nsplit > max_split) nsplit = (int)max_split;
  if (nsplit < 1) nsplit = 1;
  double* part = ensure<double>(ws.covpart, (size_t)(nsplit * d * d));
  double* A = ensure<double>(ws.A0, (size_t)m * m);
  HIPCHK(launch_covariance(p.X, p.n, d, p.mu, part, nsplit, A, m, st));
  return A;
}

// FP64 centred copy of the non-constant columns (n x dx, row-major), made
// on first use in a call.
// Rows are zero-padded to a multiple of 4096 (zero rows add nothing to the
// products; the covariance splits the rows into equal blocks).
static int64_t rows64(const Points& p) { return round_up(p.n, 4096); }
static const double* centred64(Workspace& ws, const Points& p, hipStream_t st) {
  if (!p.xc64) {
    const int64_t D = std::max<int64_t>(p.dx, 1), np = rows64(p);
    p.xc64 = ensure<double>(ws.xc64, (size_t)(np * D));
    if (p.dx > 0) HIPCHK(launch_center64(p.X, p.n, p.d, p.mu, p.colmap, p.dx, p.xc64, st));
    if (np > p.n) HIPCHK(hipMemsetAsync(p.xc64 + p.n * D, 0, sizeof(double) * (size_t)((np - p.n) * D), st));
  }
  return p.xc64;
}

// The covariance of the non-constant coordinates, C = Xc^T Xc over the FP64
// centred rows (k_dgemm), in full into ws.A0 (m_pad x m_pad, zero padding).
static double* covariance64(Workspace& ws, const Points& p, int m_pad, hipStream_t st) {
  const int64_t D = p.dx;
  double* A = ensure<double>(ws.A0, (size_t)m_pad * m_pad);
  const double* xc = centred64(ws, p, st);
  // Split-K over row blocks so that a small D still fills the GPU (about
  // 2048 workgroups, at least 256 rows each): each block gives the upper
  // tiles of a partial A_b^T A_b, and k_cov_reduce adds the partials in
  // block order and mirrors one triangle, so C is exactly symmetric.
  const int64_t np = rows64(p);
  const int64_t T = (D + dgemm_tile() - 1) / dgemm_tile();
  const int64_t tiles = T * (T + 1) / 2;
  const int64_t nsplit = std::max<int64_t>(1, std::min<int64_t>(np / 256, (2048 + tiles - 1) / tiles));
  double* part = ensure<double>(ws.covpart, (size_t)(nsplit * D * D));
  HIPCHK(launch_dgemm_syrk_upper(xc, D, D, np, (int)nsplit, part, st));
  HIPCHK(launch_cov_reduce(part, (int)nsplit, D, m_pad, A, st));
  return A;
}

// The covariance over all d coordinates (the randomized PCA's input), m x m
// with zero padding: without constant coordinates the FP64 SYRK of the
// centred rows (covariance64, about twice as fast at d = 4096), with them
// the kernel over all d columns of the FP32 rows (covariance).
static const double* full_covariance(Workspace& ws, const Points& p, int m, hipStream_t st) {
  return p.dx == p.d ? covariance64(ws, p, m, st) : covariance(ws, p, m, st);
}

// FP64 images of the principal axes that lead a fit's maps: the first s rows
// of every map the search builds (s = r/2 for Algorithm 1's maps, r for the
// PCA family) are the same FP32 copies of the rows of Vt, so their images
// (X - mu) Vt_s^T are computed once, for the largest s asked so far, and each
// probe's FP64 product covers only its other rows.  The k_dgemm result of an
// entry depends only on its row of X and its row of the map (the same k
// order at any tile position), so the images are the ones a whole product
// would give, bit for bit.  Valid while the axes stay; reset when they change
// (the randomized PCA's larger blocks).
struct AxisImages {
  double* Y = nullptr;   // n x cap, row-major; columns [0, s) hold images
  int64_t cap = 0, s = 0;
};
constexpr size_t kAxisImagesMaxBytes = (size_t)16 << 30;

// Y64 = (X - mu) Pi^T in FP64 over the non-constant columns (constant ones
// centre to exact zeros), a k_dgemm product of the FP64 centred rows and the
// FP64 values of the FP32 map.  Y64: n x r row-major.  With ai, the first
// `lead` rows of Pi are the axes behind ai and their images come from it.
static void embed64(Workspace& ws, const Points& p, const float* Pi, int64_t r, double* Y64, hipStream_t st,
                    AxisImages* ai = nullptr, int64_t lead = 0) {
  if (p.dx == 0) {
    HIPCHK(hipMemsetAsync(Y64, 0, sizeof(double) * (size_t)(p.n * r), st));
    return;
  }
  const double* xc = centred64(ws, p, st);
  double* P64 = ensure<double>(ws.pi64c, (size_t)(r * p.dx));
  HIPCHK(launch_cols64(Pi, r, p.d, p.colmap, p.dx, P64, st));
  // Y64[i][a] = sum_c xc[i][c] P64[a][c]  (P64: r x dx row-major)
  int64_t s = 0;
  if (ai && ai->Y) {
    s = std::min(std::min(lead, r), ai->cap);
    if (s > ai->s) {   // the axes' images [ai->s, s) join the kept ones
      HIPCHK(launch_dgemm_nt(xc, p.dx, P64 + ai->s * p.dx, p.dx, p.n, s - ai->s, p.dx, ai->Y + ai->s, ai->cap, st));
      ai->s = s;
    }
    HIPCHK(launch_copy_block64(ai->Y, ai->cap, Y64, r, p.n, s, st));
  }
  if (r > s) HIPCHK(launch_dgemm_nt(xc, p.dx, P64 + s * p.dx, p.dx, p.n, r - s, p.dx, Y64 + s, r, st));
}

// Randomized PCA (the paper's Sec. 4.5 variant, after Halko, Martinsson &
// Tropp's randomized subspace iteration): a block of ell sign vectors Omega
// (counter signs of the stream seed ^ kRpcaStream), Y = C Omega, then q times
// Y = C Q with Q an orthonormal basis of the previous block, and the
// Rayleigh-Ritz step on the last basis: the eigenpairs of Q^T C Q give ell
// approximate principal directions (rows of Vt_out, decreasing value) and
// values.  Bases are kept as rows (Q^T, ell x d); an orthonormal basis of a
// block Y^T is Lambda^-1/2 V^T Y^T with Y^T Y = V Lambda V^T from the Jacobi
// solver, applied twice (directions below 1e-24 of the largest are dropped).
static const uint64_t kRpcaStream = 0x94D049BB133111EBull;
static void randomized_axes(Workspace& ws, const double* C, int m, int64_t d, int64_t ell, int q, uint64_t seed,
                            double* lam_out, double* Vt_out, hipStream_t st) {
  const int mg = (int)round_up(ell, 2 * bj_block());
  double* Qt = ensure<double>(ws.rpQ, (size_t)(ell * d));
  double* Yt = ensure<double>(ws.rpY, (size_t)(ell * d));
  double* G = ensure<double>(ws.rpG, (size_t)mg * mg);
  double* V = ensure<double>(ws.rpV, (size_t)(ell * ell));
  double* lam = ensure<double>(ws.rpLam, (size_t)ell);
  auto orthonormal_rows = [&](double* src, double* dst) {   // dst = orth basis of the rows of src
    HIPCHK(launch_gram_rows(src, (int)ell, d, G, mg, st));
    jacobi_eig(ws, G, mg, ell, lam, V, st);
    HIPCHK(launch_gemm_nn(V, ell, ell, ell, src, d, d, dst, d, st));
    HIPCHK(launch_scale_rows_isqrt(dst, ell, d, lam, 1e-24, st));
  };
  HIPCHK(launch_jl_signs(seed ^ kRpcaStream, ell, d, Qt, st));            // Omega^T
  for (int it = 0; it <= q; ++it) {
    HIPCHK(launch_gemm_nt(Qt, ell, d, d, C, d, m, Yt, d, st));             // Y^T = Q^T C (C symmetric)
    orthonormal_rows(Yt, Qt);
    orthonormal_rows(Qt, Yt);
    std::swap(Qt, Yt);
  }
  // Rayleigh-Ritz: B = Q^T C Q, its eigenvectors rotate the basis
  HIPCHK(launch_gemm_nt(Qt, ell, d, d, C, d, m, Yt, d, st));               // Z^T = Q^T C
  HIPCHK(hipMemsetAsync(G, 0, sizeof(double) * (size_t)mg * mg, st));
  HIPCHK(launch_gemm_nt(Yt, ell, d, d, Qt, ell, d, G, mg, st));           // B = Z^T Q
  jacobi_eig(ws, G, mg, ell, lam_out, V, st);
  HIPCHK(launch_gemm_nn(V, ell, ell, ell, Qt, d, d, Vt_out, d, st));
}

// after_cov (optional) runs once the covariance is queued on st, before the
// eigensolver.
static Axes principal_axes(Workspace& ws, const Points& p, hipStream_t st, double* lam_out = nullptr,
                           double* Vt_out = nullptr, const std::function<void()>& after_cov = {}) {
  const int64_t d = p.d;
  // block Jacobi works on m = d rounded up to a multiple of two index blocks
  Axes ax;
  ax.lam = lam_out ? lam_out : ensure<double>(ws.lam, (size_t)d);
  ax.Vt = Vt_out ? Vt_out : ensure<double>(ws.Vt, (size_t)(d * d));
  if (p.dx == d) {
    const int m = (int)round_up(d, 2 * bj_block());
    double* A = covariance64(ws, p, m, st);
    if (after_cov) after_cov();
    ax.sweeps = jacobi_eig(ws, A, m, d, ax.lam, ax.Vt, st);
    return ax;
  }
  // Coordinates that hold one value over the cloud (listed after the others
  // in p.colmap) split off an exactly zero block of C: the eigensolver runs
  // on the covariance of the others only.
  const int64_t d1 = p.dx;
  double* lam1 = ensure<double>(ws.lam1, (size_t)std::max<int64_t>(d1, 1));
  double* Vt1 = ensure<double>(ws.Vt1, (size_t)std::max<int64_t>(d1, 1) * std::max<int64_t>(d1, 1));
  ax.sweeps = 0;
  if (d1 > 0) {
    const int m1 = (int)round_up(d1, 2 * bj_block());
    double* A1 = covariance64(ws, p, m1, st);
    if (after_cov) after_cov();
    ax.sweeps = jacobi_eig(ws, A1, m1, d1, lam1, Vt1, st);
  } else if (after_cov) {
    after_cov();
  }
  const int* idx = p.colmap;
  HIPCHK(launch_scatter_axes(lam1, Vt1, idx, (int)d1, (int)d, ax.lam, ax.Vt, st));
  return ax;
}

// ------------------------------------------------------------ learned form
static const int kSketchRows = 128;
static const uint64_t kSketchStream = 0xD1B54A32D192ED03ull;

// Features of the learned search (80 floats, device): spectrum of the JL
// sketch G = Omega Xc (kSketchRows x d, Omega = +-1/sqrt(m) signs from the
// sketch stream of `seed`), log n, log d, eps.
static void sketch_features(Workspace& ws, const Points& p, double eps, uint64_t seed, float* feat, hipStream_t st) {
  const int m = kSketchRows;
  int nsplit = (int)std::min<int64_t>(64, (p.n + 1023) / 1024);
  if (nsplit < 1) nsplit = 1;
  double* part = ensure<double>(ws.skpart, (size_t)nsplit * m * p.d);
  double* G = ensure<double>(ws.skG, (size_t)m * p.d);
  HIPCHK(launch_sketch(p.X, p.n, p.d, p.mu, m, seed ^ kSketchStream, part, nsplit, G, st));
  const int mp = (int)round_up(m, 2 * bj_block());
  double* K = ensure<double>(ws.skK, (size_t)mp * mp);
  HIPCHK(launch_gram_rows(G, m, p.d, K, mp, st));
  // eigenvalues only (the features need no eigenvectors)
  double* lam = ensure<double>(ws.sklam, (size_t)m);
  HIPCHK(launch_sym_eigvals(K, m, mp, lam, st));
  HIPCHK(launch_sketch_features(lam, m, p.n, p.d, eps, feat, st));
}

struct MlpBufs {
  __bf16* pb;
  __bf16* X;
  MlpActs a;
  float* out;
};

static MlpBufs mlp_bufs(Workspace& ws, const MlpLayout& L, int B) {
  MlpBufs b;
  b.pb = ensure<__bf16>(ws.mlp_pb, (size_t)L.total);
  b.X = ensure<__bf16>(ws.mlp_X, (size_t)B * L.in_pad);
  const size_t BH = (size_t)B * L.hidden;
  float* f = ensure<float>(ws.mlp_f, 5 * BH + 2 * (size_t)B);
  b.a.A1 = f;
  b.a.A2 = f + BH;
  b.a.A3 = f + 2 * BH;
  b.a.dZ = f + 3 * BH;
  b.a.dZ2 = f + 4 * BH;
  b.a.g = f + 5 * BH;
  b.out = f + 5 * BH + B;
  __bf16* hb = ensure<__bf16>(ws.mlp_hb, 2 * BH);
  b.a.A1b = hb;
  b.a.A2b = hb + BH;
  return b;
}

// Predicted log(r / d) for one feature row (host float).
static float mlp_predict(Workspace& ws, const float* params, const float* feat, hipStream_t st) {
  const MlpLayout L = mlp_layout();
  MlpBufs b = mlp_bufs(ws, L, 1);
  HIPCHK(mlp_to_bf16(params, b.pb, L.total, st));
  HIPCHK(mlp_to_bf16(feat, b.X, L.in_pad, st));
  HIPCHK(mlp_forward(L, params, b.pb, b.X, 1, b.a, b.out, st));
  float h = 0.0f;
  HIPCHK(hipMemcpyAsync(&h, b.out, sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return h;
}

// ------------------------------------------------------------------ map
// Pi (r x d, FP32) of Algorithm 1 at target dimension r.
static void build_map(Workspace& ws, const double* Vt, int64_t d, int64_t r, uint64_t seed, float* Pi,
                      hipStream_t st) {
  if (r == d) {
    HIPCHK(launch_copy_rows(Vt, d, d, Pi, nullptr, st));
    return;
  }
  const int64_t s = r / 2, k = r - r / 2;
  HIPCHK(launch_copy_rows(Vt, s, d, Pi, nullptr, st));
  double* S = ensure<double>(ws.S, (size_t)(k * d));
  HIPCHK(launch_jl_signs(seed, k, d, S, st));
  double* T = ensure<double>(ws.T, (size_t)(k * (s > 0 ? s : 1)));
  if (s > 0) HIPCHK(launch_proj_T(S, k, d, Vt, s, T, st));
  HIPCHK(launch_proj_SQ(S, T, k, s, Vt, d, Pi, nullptr, st));
}

// Pi (r x d, FP32) of a map family at target dimension r: Algorithm 1, the
// top r principal directions alone, or Lemma 1's JL matrix alone (r = d: the
// identity, no reduction).
static void build_family_map(Workspace& ws, int family, const double* Vt, int64_t d, int64_t r, uint64_t seed,
                             float* Pi, hipStream_t st) {
  if (family == ADAGIO_MAP_PCA) {
    HIPCHK(launch_copy_rows(Vt, r, d, Pi, nullptr, st));
  } else if (family == ADAGIO_MAP_JL) {
    double* S = ensure<double>(ws.S, (size_t)(r * d));
    if (r == d) HIPCHK(launch_eye(S, (int)d, st));
    else HIPCHK(launch_jl_signs(seed, r, d, S, st));
    HIPCHK(launch_copy_rows(S, r, d, Pi, nullptr, st));
  } else {
    build_map(ws, Vt, d, r, seed, Pi, st);
  }
}

// ----------------------------------------------------------- certificate
struct Images {
  int64_t r = 0, ldy = 0;
  int64_t rs = 0;               // columns of the screen images Yc: r, or d' for images through the Gram factor
  float* Yc = nullptr;
  float2* ty = nullptr;
  int64_t ldyb = 0;             // BF16 split (screen = BF16X3)
  __bf16* Yb = nullptr;
  float2* tyb = nullptr;
  int64_t ldyq = 0;             // per-row scaled e4m3 copy (screen = FP8)
  unsigned char* Yq = nullptr;
  float4* q8 = nullptr;         // per row (N_x, N_y, -2 s_x, -2 s_y) of the FP8 screen
  const float* Y32 = nullptr;   // rescore source (given images) ...
  const double* Y64 = nullptr;  // ... or FP64 images of a map
};

// The screen's reduced-precision copies of the centred images Yc (row norms
// ny); nx_emb / c_emb: the FP64 embedding error term of images of a map.
static void image_copies(Workspace& ws, const Points& p, Images& im, const double* ny, const double* nx_emb,
                         double c_emb, hipStream_t st) {
  if (p.screen == ADAGIO_SCREEN_BF16X3 || p.screen == ADAGIO_SCREEN_FP8) {
    im.ldyb = round_up(im.rs, kChunkBf16);
    im.Yb = ensure<__bf16>(ws.Yb, (size_t)(p.n_pad * 2 * im.ldyb));
    im.tyb = ensure<float2>(ws.tyb, (size_t)p.n_pad);
    HIPCHK(launch_split_bf16(im.Yc, p.n_pad, im.rs, im.ldy, im.ldyb, im.Yb, st));
    HIPCHK(launch_row_terms(ny, screen_const_bf16(im.ldyb), nx_emb, c_emb, p.n_pad, im.tyb, st));
  }
  if (p.screen == ADAGIO_SCREEN_FP8) {
    im.ldyq = round_up(im.rs, fp8_chunk());
    im.Yq = ensure<unsigned char>(ws.Yq, (size_t)(p.n_pad * im.ldyq));
    float* sy = ensure<float>(ws.sy, (size_t)p.n_pad);
    double* nyq = ensure<double>(ws.nyq, (size_t)p.n_pad);
    HIPCHK(launch_quant_fp8(im.Yc, p.n_pad, im.rs, im.ldy, im.ldyq, im.Yq, sy, nyq, st));
    im.q8 = ensure<float4>(ws.q8terms, (size_t)p.n_pad);
    HIPCHK(launch_fp8_terms(p.xgram_split ? p.nx : p.nxq, nyq, p.xgram_split ? nullptr : p.sx, sy, p.n_pad, im.q8,
                            st));
  }
}

// Screen images through the Gram factor, for a map with r >= d' + 32 rows
// (d' non-constant coordinates): M = Pi'^T Pi' (d' x d', FP64 k_dgemm over
// the FP64 values of Pi's columns), M = L L^T (k_cholesky), and
// Z = (X - mu)' L (n x d', FP64 k_dgemm).  ||z_i - z_j||^2 = v^T L L^T v
// for the difference v of the non-constant coordinates, and
// |v^T L L^T v - v^T M v| <= (gamma_r + 1.01 gamma_{d'+1}) ||Pi||_F^2 ||v||^2
// (the dot products of M, then the factor's backward error).  Null when
// d' is beyond the factor kernel's size or the factor fails (then the
// screen takes the r images).
static double* gram_factor_images(Workspace& ws, const Points& p, int64_t r, hipStream_t st) {
  const int64_t m = p.dx;
  if (m < 1 || m > chol_max_m() || r < m + 32) return nullptr;
  const double* P64 = static_cast<const double*>(ws.pi64c.p);   // r x m, row-major, from embed64
  double* M = ensure<double>(ws.gfM, (size_t)(m * m));
  int* fail = ensure<int>(ws.gfFail, 1);
  // M[c][c'] = sum_a P64[a][c] P64[a][c'] (symmetric: row- and column-major alike)
  HIPCHK(launch_dgemm_tn(P64, m, P64, m, m, m, r, 1, M, m, st));
  HIPCHK(hipMemsetAsync(fail, 0, sizeof(int), st));
  HIPCHK(launch_cholesky(M, (int)m, fail, st));
  int hf = 0;
  HIPCHK(hipMemcpyAsync(&hf, fail, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hf) return nullptr;
  const double* xc = centred64(ws, p, st);
  double* Z = ensure<double>(ws.gfZ, (size_t)(p.n * m));
  // Z[i][j] = sum_c xc[i][c] L[c][j], L column-major in M: L[c][j] = M[j * m + c]
  HIPCHK(launch_dgemm_nt(xc, m, M, m, p.n, m, m, Z, m, st));
  return Z;
}

// Images of the linear map Pi in FP64, centred: Y64 = (X - mu) Pi^T (the
// re-evaluation source), and the screen images: Y64 itself, or Z from the
// Gram factor when Pi has at least d' + 32 rows.
static Images images_of_map(Workspace& ws, const Points& p, const float* Pi, int64_t r, hipStream_t st,
                            AxisImages* ai = nullptr, int64_t lead = 0) {
  Images im;
  im.r = r;
  double* Y64 = ensure<double>(ws.Y64, (size_t)(p.n * r));
  embed64(ws, p, Pi, r, Y64, st, ai, lead);
  // FP64 embedding error: |E_64^2 - E^2| <= 4.02 gamma_{d'+1} ||Pi'||_F^2 (N_i + N_j)
  // over the d' non-constant coordinates (and ||L||_F^2 = trace(M) <=
  // ||Pi'||_F^2 for the factor's images); ||Pi'||_F^2 from the FP64 values of
  // Pi's columns (a sum of squares, inflated far beyond its rounding).
  double pf2 = 0.0;
  if (p.dx > 0) {
    const int nparts = 256;
    double* part = ensure<double>(ws.nrm, nparts + 1);
    HIPCHK(launch_sumsq(static_cast<const double*>(ws.pi64c.p), p.dx * r, part, nparts, part + nparts, st));
    HIPCHK(hipMemcpyAsync(&pf2, part + nparts, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    pf2 *= 1.0 + 1e-8;
  }
  const double dx1 = (double)p.dx + 1.0;
  double c_emb = 4.02 * pf2 * dx1 * kU64 * 1.01;
  const double* Ys = Y64;
  im.rs = r;
  if (const double* Z = gram_factor_images(ws, p, r, st)) {
    Ys = Z;
    im.rs = p.dx;
    // ||v||^2 <= 2 (N_i + N_j)
    c_emb += 2.0 * pf2 * ((double)r + 1.01 * dx1) * kU64 * 1.01;
  }
  im.ldy = round_up(im.rs, kChunk);
  im.Yc = ensure<float>(ws.Yc, (size_t)(p.n_pad * im.ldy));
  double* ny = ensure<double>(ws.ny, (size_t)p.n_pad);
  HIPCHK(launch_center<double>(Ys, p.n, im.rs, im.rs, nullptr, im.Yc, im.ldy, p.n_pad, ny, st));
  im.ty = ensure<float2>(ws.ty, (size_t)p.n_pad);
  HIPCHK(launch_row_terms(ny, screen_const(im.ldy), p.nx, c_emb, p.n_pad, im.ty, st));
  image_copies(ws, p, im, ny, p.nx, c_emb, st);
  im.Y64 = Y64;
  return im;
}

// Given images (FP32), centred by their own mean.
static Images images_given(Workspace& ws, const Points& p, const float* Y, int64_t r, hipStream_t st) {
  Images im;
  im.r = r;
  im.rs = r;
  im.ldy = round_up(r, kChunk);
  double* muY = ensure<double>(ws.muY, (size_t)r);
  mean_rows(ws, Y, p.n, r, r, muY, st);
  im.Yc = ensure<float>(ws.Yc, (size_t)(p.n_pad * im.ldy));
  double* ny = ensure<double>(ws.ny, (size_t)p.n_pad);
  HIPCHK(launch_center<float>(Y, p.n, r, r, muY, im.Yc, im.ldy, p.n_pad, ny, st));
  im.ty = ensure<float2>(ws.ty, (size_t)p.n_pad);
  HIPCHK(launch_row_terms(ny, screen_const(im.ldy), nullptr, 0.0, p.n_pad, im.ty, st));
  image_copies(ws, p, im, ny, nullptr, 0.0, st);
  im.Y32 = Y;
  return im;
}

struct CertTimes {
  double screen_ms = 0.0, rest_ms = 0.0;
  int64_t flagged = 0, rescored = 0;
  int screened = 0;   // FP8 screens among the calls
  int nprobe = 0;
  int refuted = 0;    // probes refuted by a witness pair
  int32_t probe_r[48], probe_cols[48];
  double probe_delta[48], probe_ms[48];
  int32_t probe_gram[48];
};

static void log_probe(CertTimes& tm, int64_t r, int64_t cols, const adagio_cert_t& c, double screen_ms, int gmode) {
  if (tm.nprobe < 48) {
    tm.probe_r[tm.nprobe] = (int32_t)r;
    tm.probe_cols[tm.nprobe] = (int32_t)cols;
    tm.probe_delta[tm.nprobe] = c.max_distortion;
    tm.probe_ms[tm.nprobe] = screen_ms;
    tm.probe_gram[tm.nprobe] = gmode;
    ++tm.nprobe;
  }
}

static void fill_stats(adagio_stats_t* s, const CertTimes& tm, int ncert, double total_ms) {
  memset(s, 0, sizeof(*s));
  s->t_screen_ms = tm.screen_ms;
  s->t_rescore_ms = tm.rest_ms;
  s->n_certificates = ncert;
  s->n_flagged_tiles = tm.flagged;
  s->n_rescored = tm.rescored;
  s->n_probes = tm.nprobe;
  s->n_screened = tm.screened;
  for (int k = 0; k < tm.nprobe; ++k) {
    s->probe_r[k] = tm.probe_r[k];
    s->probe_delta[k] = tm.probe_delta[k];
    s->probe_screen_ms[k] = tm.probe_ms[k];
    s->probe_gram[k] = tm.probe_gram[k];
    s->probe_cols[k] = tm.probe_cols[k];
  }
  s->n_refuted = tm.refuted;
  s->t_total_ms = total_ms;
}

static void rescore(const Points& p, const Images& im, const int2* pairs, const uint32_t* count_ptr,
                    const int* count_i, uint32_t cap, PairVal* out, int grid, hipStream_t st) {
  if (im.Y64) HIPCHK(launch_rescore<double>(p.X, p.d, im.Y64, im.r, pairs, count_ptr, count_i, cap, out, grid, st));
  else HIPCHK(launch_rescore<float>(p.X, p.d, im.Y32, im.r, pairs, count_ptr, count_i, cap, out, grid, st));
}

// Witness pool of a fit's search (record pairs of earlier certificates) and
// the margin above eps that a witness must clear.
static const uint32_t kPoolCap = 16384;
static const uint32_t kPoolTiles = 256;
static const double kWitnessMargin = 1e-9;

static const uint32_t kDefaultCap = 1u << 20;
static const uint32_t kHardCap = 1u << 26;
// FP8 screen: tiles re-screened with the FP32 bounds (at most 4x that many
// when key buckets tie).
static const uint32_t kFp8Tiles = 1024;

// Largest eigensolver size (m, the padded covariance order) that a fit's
// cache fill runs beside: at m = 832 the fill (8 ms) hides beside the PCA
// (7 -> 10 ms); at m = 4096 the sweeps it overlapped took 76 ms each and the
// overlap gained nothing.
static const int64_t kFillBesideMaxM = 1024;

// Point-Gram cache for the certificates of one fit: the points do not change
// across a fit's certificates, so a fill stores every tile's point side once
// and the screens read it back instead of recomputing it.  FP32 screens keep
// the FP32 point Gram (64 KB per tile of pairs), the precision forms the
// compact D^2 cache (32 KB per tile).  Null (no caching) when it would take
// more than half of the free device memory.
static float* gram_cache(Workspace& ws, const Points& p) {
  const int64_t NT = p.n_pad / kTile;
  const bool compact = p.screen == ADAGIO_SCREEN_BF16X3 || p.screen == ADAGIO_SCREEN_FP8;
  const size_t per_tile = compact ? (size_t)kDcacheBytesPerTile : (size_t)kGcacheFloatsPerTile * sizeof(float);
  const size_t bytes = (size_t)(NT * (NT + 1) / 2) * per_tile;
  if (ws.gcache.cap >= bytes) return static_cast<float*>(ws.gcache.p);
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return nullptr;
  if (bytes > (fr + ws.gcache.cap) / 2) return nullptr;
  return ensure<float>(ws.gcache, bytes / sizeof(float));
}

// A probe refuted by a witness pair: kind 3 from the pool (no screen), 4 from
// a screen that stopped early (screen_ms: its partial time).
static void log_refuted(CertTimes& tm, int64_t r, int64_t cols, double w, int kind, double screen_ms) {
  ++tm.refuted;
  if (tm.nprobe < 48) {
    tm.probe_r[tm.nprobe] = (int32_t)r;
    tm.probe_cols[tm.nprobe] = (int32_t)cols;
    tm.probe_delta[tm.nprobe] = w;
    tm.probe_ms[tm.nprobe] = screen_ms;
    tm.probe_gram[tm.nprobe] = kind;
    ++tm.nprobe;
  }
}

// Early stop of a fit's screen: the screen records pairs whose bounds prove
// eq. (2) > eps + 2e-9 and stops; one of them re-evaluated above
// eps + kWitnessMargin fails the probe.
struct StopOut {
  bool stopped = false;
  PairVal w;
};

static float f32_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = nextafterf(f, INFINITY);
  return f;
}
static float f32_down(double x) {
  float f = (float)x;
  if ((double)f > x) f = nextafterf(f, -INFINITY);
  return f;
}

// The certificate of eq. (3) for points p and images im.  With the FP8 screen
// the same steps run on the FP8 estimates' top tiles only, and the result is
// the exact maximum over those tiles (certified = 0, no bound on the rest).
// grow = false: the candidate buffer keeps capacity cap0 (a fixed arena);
// more candidates than that leave the certificate incomplete.
static adagio_cert_t certificate(Workspace& ws, const Points& p, const Images& im, uint32_t cap0,
                                 hipStream_t st, CertTimes* times, int screen, float* gcache = nullptr,
                                 int gmode = 0, double stop_eps = -1.0, StopOut* so = nullptr,
                                 bool grow = true) {
  PairsView v;
  v.X = p.Xc; v.ldx = (int)p.ldx;
  v.Y = im.Yc; v.ldy = (int)im.ldy;
  v.tx = p.tx; v.ty = im.ty;
  v.n = (int)p.n;
  v.NT = (int)(p.n_pad / kTile);
  v.ntiles = (int64_t)v.NT * (v.NT + 1) / 2;

  TileRec* recs = ensure<TileRec>(ws.recs, (size_t)v.ntiles);
  const int nparts = 256;
  TileRec* tparts = ensure<TileRec>(ws.tparts, nparts + 1);
  int2* seeds = ensure<int2>(ws.seeds, 2);
  PairVal* seedv = ensure<PairVal>(ws.seedv, 2);
  uint32_t* list = ensure<uint32_t>(ws.list, (size_t)v.ntiles);
  CertDev* cd = ensure<CertDev>(ws.cd, 1);
  const int vp = 64;
  PairVal* vparts = ensure<PairVal>(ws.vparts, 2 * vp);

  ScreenStop ss;
  const ScreenStop* sp = nullptr;
  if (stop_eps > 0.0 && so && screen != ADAGIO_SCREEN_FP8 && gmode != 1) {
    const double e = stop_eps + 2.0 * kWitnessMargin;
    ss.count = ensure<uint32_t>(ws.stopn, 1);
    ss.pairs = ensure<int2>(ws.stopp, 8);
    ss.q_hi = f32_up((1.0 + e) * (1.0 + e));
    ss.q_lo = e < 1.0 ? f32_down((1.0 - e) * (1.0 - e)) : -1.0f;
    HIPCHK(hipMemsetAsync(ss.count, 0, sizeof(uint32_t), st));
    sp = &ss;
  }
  EvPair e_screen, e_rest;
  e_screen.on = e_rest.on = times != nullptr;
  auto run_screen = [&](const ScreenStop* stop) {
    e_screen.begin(st);
    if (screen == ADAGIO_SCREEN_BF16X3) {
      // BF16 split screen; the emit pass below keeps the FP32 Gram (tighter
      // bounds, fewer candidates, equally rigorous).
      PairsViewB vb;
      vb.Xb = p.Xb; vb.ldx = (int)p.ldxb;
      vb.Yb = im.Yb; vb.ldy = (int)im.ldyb;
      vb.tx = p.txb; vb.ty = im.tyb;
      vb.n = v.n; vb.NT = v.NT; vb.ntiles = v.ntiles;
      vb.dscale = p.dscale;
      HIPCHK(launch_pairs_screen_bf16(vb, recs, gcache, gmode, stop, st));
    } else if (screen == ADAGIO_SCREEN_FP8) {
      HIPCHK(launch_pairs_screen_fp8(p.Xq, (int)p.ldxq, im.Yq, (int)im.ldyq, im.q8, v.n, v.NT, recs, gcache, gmode,
                                     p.dscale, st));
    } else {
      HIPCHK(launch_pairs_screen(v, recs, gcache, gmode, stop, st));
    }
    e_screen.end(st);
  };
  run_screen(sp);
  if (sp) {
    uint32_t hc = 0;
    HIPCHK(hipMemcpyAsync(&hc, ss.count, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hc > 0) {
      PairVal* wv = ensure<PairVal>(ws.wvals, kPoolCap);
      PairVal* parts = ensure<PairVal>(ws.wparts, 64);
      CertDev* wcd = ensure<CertDev>(ws.wcd, 1);
      rescore(p, im, ss.pairs, ss.count, nullptr, 8, wv, 1, st);
      HIPCHK(launch_best_reset(wcd, st));
      HIPCHK(launch_top2(wv, ss.count, 8, parts, 1, wcd, st));
      PairVal w;
      HIPCHK(hipMemcpyAsync(&w, &wcd->best, sizeof(PairVal), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (w.i >= 0 && w.v > stop_eps + kWitnessMargin) {
        so->stopped = true;
        so->w = w;
        adagio_cert_t c;
        memset(&c, 0, sizeof(c));
        c.n_pairs = p.n * (p.n - 1) / 2;
        c.max_distortion = w.v;
        c.i = w.i;
        c.j = w.j;
        c.side = w.side;
        c.runner_up = -1.0;
        c.i2 = c.j2 = -1;
        c.bound_rest = INFINITY;
        if (times) {
          const double sm = e_screen.ms();
          times->screen_ms += sm;
          log_refuted(*times, im.r, im.rs, w.v, 4, sm);
        }
        return c;
      }
      // The bounds are rigorous, so this does not happen; if it did, the
      // records of the skipped tiles would be stale: screen again in full.
      run_screen(nullptr);
    }
  }
  e_rest.begin(st);
  HIPCHK(launch_seeds(recs, v.ntiles, tparts, nparts, seeds, cd, st));
  rescore(p, im, seeds, nullptr, &cd->n_seed, 2, seedv, 1, st);
  HIPCHK(launch_thresholds(seedv, cd, st));
  if (screen == ADAGIO_SCREEN_FP8) {
    uint32_t* hist = ensure<uint32_t>(ws.hist, kTopkHistWords);
    uint32_t* kthr = ensure<uint32_t>(ws.kthr, 1);
    HIPCHK(launch_topk_tiles(recs, v.ntiles, kFp8Tiles, 4 * kFp8Tiles, hist, kthr, list, &cd->n_flagged, st));
  } else {
    HIPCHK(launch_flag_tiles(recs, v.ntiles, cd, list, st));
  }

  uint32_t cap = cap0 ? cap0 : kDefaultCap;
  CertDev h;
  // When the bounds cannot separate pairs (a near-isometry: every pair's
  // bound reaches the best exact value), the flagged tiles can hold more
  // candidates than the hard cap and the exact pass would only overflow;
  // report the proven bound instead.
  HIPCHK(hipMemcpyAsync(&h, cd, sizeof(CertDev), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const bool skip_exact = (int64_t)h.n_flagged * kTile * kTile > (int64_t)kHardCap;
  if (skip_exact) h.n_cand = 0xffffffffu;
  for (; !skip_exact;) {
    int2* cand = ensure<int2>(ws.cand, cap);
    PairVal* vals = ensure<PairVal>(ws.vals, cap);
    HIPCHK(hipMemsetAsync(&cd->n_cand, 0, sizeof(uint32_t), st));
    const int egrid = (int)std::min<int64_t>(v.ntiles, 2048);
    HIPCHK(launch_pairs_emit(v, list, cd, cand, cap, &cd->n_cand, egrid, st));
    rescore(p, im, cand, &cd->n_cand, nullptr, cap, vals, 1024, st);
    HIPCHK(launch_top2(vals, &cd->n_cand, cap, vparts, vp, cd, st));
    HIPCHK(hipMemcpyAsync(&h, cd, sizeof(CertDev), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h.n_cand <= cap || cap >= kHardCap || !grow) break;
    // More candidates than room: grow and redo the exact pass (the thresholds
    // and flagged tiles are unchanged).
    cap = h.n_cand > kHardCap ? kHardCap : h.n_cand;
    // restore the seed-only best/second before re-merging
    HIPCHK(launch_thresholds(seedv, cd, st));
  }
  e_rest.end(st);
  HIPCHK(hipStreamSynchronize(st));

  adagio_cert_t c;
  memset(&c, 0, sizeof(c));
  c.n_pairs = p.n * (p.n - 1) / 2;
  c.n_flagged_tiles = h.n_flagged;
  c.n_rescored = (int64_t)h.n_seed + (skip_exact ? 0 : (int64_t)std::min<uint32_t>(h.n_cand, cap));
  const bool complete = !skip_exact && h.n_cand <= cap;
  if (h.best.i >= 0) {
    c.max_distortion = h.best.v;
    c.i = h.best.i;
    c.j = h.best.j;
    c.side = h.best.side;
  } else {
    c.max_distortion = 0.0;
    c.i = c.j = -1;
    c.side = 0;
  }
  if (h.second.i >= 0) {
    c.runner_up = h.second.v;
    c.i2 = h.second.i;
    c.j2 = h.second.j;
  } else {
    c.runner_up = -1.0;
    c.i2 = c.j2 = -1;
  }
  // Rigorous bound over every pair from the screen's global extremes.
  const double qh = (double)h.qhi_all, ql = (double)h.qlo_all;
  const double ub = std::max(std::sqrt(std::max(qh, 0.0)) - 1.0, 1.0 - std::sqrt(std::max(ql, 0.0)));
  if (screen == ADAGIO_SCREEN_FP8) {
    c.certified = 0;
    c.bound_rest = INFINITY;
  } else if (complete) {
    c.certified = 1;
    c.bound_rest = h.bound_rest;
  } else {
    c.certified = 0;
    c.bound_rest = std::max(ub * (1.0 + 1e-12), c.max_distortion);
  }
  if (times) {
    const double sm = e_screen.ms();
    times->screen_ms += sm;
    times->rest_ms += e_rest.ms();
    times->flagged += h.n_flagged;
    times->rescored += c.n_rescored;
    if (screen == ADAGIO_SCREEN_FP8) ++times->screened;
    log_probe(*times, im.r, im.rs, c, sm, gcache ? gmode : 0);
  }
  return c;
}

// Witness pool of a fit's search (eq. (3) is a maximum: one pair above eps
// fails a map).  Each certificate adds the record pairs of its kPoolTiles
// tiles of largest bound; a probe evaluates the pool exactly, by direct
// differences, before it embeds the cloud and screens it.

static void pool_reset(Workspace& ws, hipStream_t st) {
  uint32_t* pn = ensure<uint32_t>(ws.pooln, 2);
  HIPCHK(hipMemsetAsync(pn, 0, 2 * sizeof(uint32_t), st));
}

// After a certificate of points p (its tile records are still in ws.recs):
// appends the pairs and recomputes their difference rows.  Returns the pool
// size.
static uint32_t pool_add(Workspace& ws, const Points& p, hipStream_t st) {
  const int64_t NT = p.n_pad / kTile;
  const int64_t ntiles = NT * (NT + 1) / 2;
  int2* pool = ensure<int2>(ws.pool, kPoolCap);
  uint32_t* pn = static_cast<uint32_t*>(ws.pooln.p);          // [0] pool size, [1] selected tiles
  uint32_t* hist = ensure<uint32_t>(ws.hist, kTopkHistWords);
  uint32_t* kthr = ensure<uint32_t>(ws.kthr, 1);
  uint32_t* list = ensure<uint32_t>(ws.list, (size_t)ntiles);
  const TileRec* recs = static_cast<const TileRec*>(ws.recs.p);
  HIPCHK(hipMemsetAsync(pn + 1, 0, sizeof(uint32_t), st));
  HIPCHK(launch_topk_tiles(recs, ntiles, kPoolTiles, 4 * kPoolTiles, hist, kthr, list, pn + 1, st));
  HIPCHK(launch_pool_gather(recs, list, pn + 1, 4 * kPoolTiles, pool, pn, kPoolCap, st));
  uint32_t cnt = 0;
  HIPCHK(hipMemcpyAsync(&cnt, pn, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  cnt = std::min(cnt, kPoolCap);
  if (cnt > 0 && p.dx > 0) {
    double* V = ensure<double>(ws.wV, (size_t)cnt * (size_t)p.dx);
    HIPCHK(launch_pair_diffs(p.X, p.d, p.colmap, p.dx, pool, cnt, V, st));
  }
  return cnt;
}

// The largest eq. (2) value over the pool's npool pairs under the map Pi
// (r x d FP32), by direct differences: W = V Pi^T in FP64 (k_dgemm over the
// non-constant coordinates).  i < 0: no pair with x_i != x_j.
static PairVal pool_witness(Workspace& ws, const Points& p, const float* Pi, int64_t r, uint32_t npool,
                            hipStream_t st) {
  PairVal w;
  w.v = -1.0; w.i = w.j = -1; w.side = 0; w.pad = 0;
  if (npool == 0 || p.dx == 0) return w;
  const int2* pool = static_cast<const int2*>(ws.pool.p);
  const uint32_t* pn = static_cast<const uint32_t*>(ws.pooln.p);
  const double* V = static_cast<const double*>(ws.wV.p);
  double* W = ensure<double>(ws.wW, (size_t)npool * (size_t)r);
  double* P64 = ensure<double>(ws.pi64c, (size_t)(r * p.dx));
  PairVal* vals = ensure<PairVal>(ws.wvals, kPoolCap);
  const int vp = 32;
  PairVal* parts = ensure<PairVal>(ws.wparts, 2 * vp);
  CertDev* wcd = ensure<CertDev>(ws.wcd, 1);
  HIPCHK(launch_cols64(Pi, r, p.d, p.colmap, p.dx, P64, st));
  // W[q][a] = sum_c V[q][c] P64[a][c]  (npool x r)
  HIPCHK(launch_dgemm_nt(V, p.dx, P64, p.dx, npool, r, p.dx, W, r, st));
  HIPCHK(launch_pair_ratio(V, p.dx, W, r, pool, npool, vals, st));
  HIPCHK(launch_best_reset(wcd, st));
  HIPCHK(launch_top2(vals, pn, npool, parts, vp, wcd, st));
  HIPCHK(hipMemcpyAsync(&w, &wcd->best, sizeof(PairVal), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return w;
}

static hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// The library's two extra streams, both of default priority.  aux runs the
// point-Gram fill on 7/8 of the CUs (a CU-masked stream, so that the PCA's
// small latency-bound kernels keep CUs of their own; a plain non-blocking
// stream if the mask is refused).  A CU-masked stream is a blocking stream:
// it orders itself after work on the null stream, and later null-stream work
// after it, so the PCA beside it runs on aux2, non-blocking.  Both are the
// device's (g_aux, g_aux2), made once and kept until the process ends.
static void ensure_streams(Workspace& ws) {
  if (!ws.aux || !ws.aux2) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));   // 0 <= dev < 64: checked when the call began
    if (!g_aux[dev]) {
      int ncu = 0;
      HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
      const int keep = ncu - ncu / 8;
      std::vector<uint32_t> mask((size_t)(ncu + 31) / 32, 0u);
      for (int c = 0; c < keep; ++c) mask[(size_t)c / 32] |= 1u << (c % 32);
      hipStream_t q = nullptr;
      if (ncu < 16 || hipExtStreamCreateWithCUMask(&q, (uint32_t)mask.size(), mask.data()) != hipSuccess) {
        (void)hipGetLastError();
        q = nullptr;
        HIPCHK(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
      }
      g_aux[dev] = q;
      if (!g_exit_hook) g_exit_hook = atexit(release_at_exit) == 0;
    }
    if (!g_aux2[dev]) {
      hipStream_t q = nullptr;
      HIPCHK(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
      g_aux2[dev] = q;
      if (!g_exit_hook) g_exit_hook = atexit(release_at_exit) == 0;
    }
    ws.aux = g_aux[dev];
    ws.aux2 = g_aux2[dev];
  }
  for (hipEvent_t* e : {&ws.ev_in, &ws.ev_out, &ws.ev_pca, &ws.ev_cov}) {
    if (!*e) HIPCHK(hipEventCreateWithFlags(e, hipEventDisableTiming));
  }
  for (hipEvent_t* e : {&ws.ev_t0, &ws.ev_t1}) {
    if (!*e) HIPCHK(hipEventCreate(e));
  }
}

// Point Gram of every tile into the fit's cache, on ws.aux (CU-masked, to
// run beside other work) or, with `alone`, on ws.aux2 (all CUs,
// non-blocking), after the work already queued on `after` (at least the
// centred copies; in a fit with the exact PCA also its covariance, or the
// whole PCA); the caller's stream waits for it with ws.ev_out before its
// first screen.  The points' Gram does not depend on the map, so it can
// overlap the PCA's eigensolver where that leaves most of the GPU idle.  The
// fill's kernel time is read later from ws.ev_t0 / ev_t1.
static void gram_fill_async(Workspace& ws, const Points& p, int screen, float* gcache, hipStream_t after,
                            bool alone = false) {
  ensure_streams(ws);
  const hipStream_t q = alone ? ws.aux2 : ws.aux;
  HIPCHK(hipEventRecord(ws.ev_cov, after));
  HIPCHK(hipStreamWaitEvent(q, ws.ev_cov, 0));
  HIPCHK(hipEventRecord(ws.ev_t0, q));
  const int NT = (int)(p.n_pad / kTile);
  const int64_t ntiles = (int64_t)NT * (NT + 1) / 2;
  if (screen == ADAGIO_SCREEN_BF16X3 || screen == ADAGIO_SCREEN_FP8) {
    // the compact D^2 cache, from the BF16 split point Gram: an FP8 fit's
    // screens and its BF16 split certificates share this one
    HIPCHK(launch_dcache_scale(p.nx, p.n_pad, p.dscale, q));
    PairsViewB vb;
    vb.Xb = p.Xb; vb.ldx = (int)p.ldxb;
    vb.Yb = p.Xb; vb.ldy = 0;
    vb.tx = p.txb; vb.ty = p.txb;
    vb.n = (int)p.n; vb.NT = NT; vb.ntiles = ntiles;
    vb.dscale = p.dscale;
    HIPCHK(launch_pairs_gram_fill_bf16(vb, gcache, q));
  } else {
    PairsView v;
    v.X = p.Xc; v.ldx = (int)p.ldx;
    v.Y = p.Xc; v.ldy = 0;
    v.tx = p.tx; v.ty = p.tx;
    v.n = (int)p.n; v.NT = NT; v.ntiles = ntiles;
    HIPCHK(launch_pairs_gram_fill(v, gcache, q));
  }
  HIPCHK(hipEventRecord(ws.ev_t1, q));
  HIPCHK(hipEventRecord(ws.ev_out, q));
}

template <typename F>
static int guarded(F&& f) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_err.clear();
  try {
    f();
    return ADAGIO_OK;
  } catch (const Fail& e) {
    return e.code;
  } catch (...) {
    g_err = "unexpected host exception";
    return ADAGIO_E_HIP;
  }
}

// Launch geometry bounds the sizes: a dispatch holds fewer than 2^32
// work-items, the all-pairs screens run one 256-thread workgroup per tile
// slot (n = 700000 gives 1.5e7 slots, 3.8e9 work-items; 740352 points would
// reach 2^32), and the elementwise kernels one work-item per element of an
// n x d copy or a d x d matrix.
static const int64_t kMaxPoints = 700000;
static const int64_t kMaxDim = 32768;

// Scratch of adagio_max_distortion_noalloc: a fixed device array (one copy
// on each GPU the library runs on, held until the process ends).  Host code
// uses its device address from hipGetSymbolAddress, taken once per device
// with that device current; the array's name is only a host-side stand-in.
static const size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static void* g_scratch[64];
// candidate pairs the scratch must leave room for beyond the fixed buffers
static const uint32_t kScratchMinCand = 1u << 16;

static void* scratch_ptr(int dev) {
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch[dev] = ptr;
  }
  return g_scratch[dev];
}

// Bytes the FP32-screen certificate of n points (d coordinates) and r image
// coordinates carves from an arena before its candidate buffers: every
// buffer of prep_points, images_given and certificate, each rounded up to
// 256 bytes (an upper bound: the screens' copies may have fewer columns).
static size_t noalloc_fixed_bytes(int64_t n, int64_t d, int64_t r) {
  const int64_t n_pad = round_up(n, kTile), nch = (n + 511) / 512;
  const int64_t ldx = round_up(d, kChunk), ldy = round_up(r, kChunk);
  const int64_t NT = n_pad / kTile, ntiles = NT * (NT + 1) / 2;
  const int64_t sizes[] = {
      d * 8, d * 4, nch * d * 8, 2 * 4, 2 * nch * d * 8, d * 4,              // mu, colmap, mean_rows(X)
      n_pad * ldx * 4, n_pad * 8, n_pad * 8,                                  // Xc, nx, tx
      r * 8, nch * r * 8, n_pad * ldy * 4, n_pad * 8, n_pad * 8,              // muY, mean_rows(Y), Yc, ny, ty
      ntiles * (int64_t)sizeof(TileRec), 257 * (int64_t)sizeof(TileRec), 2 * 8,  // recs, tparts, seeds
      2 * (int64_t)sizeof(PairVal), ntiles * 4, (int64_t)sizeof(CertDev),     // seedv, list, cd
      128 * (int64_t)sizeof(PairVal)};                                        // vparts
  size_t tot = 0;
  for (int64_t b : sizes) tot += (size_t)round_up(std::max<int64_t>(b, 1), 256) + 256;
  return tot;
}

static void check_points(const float* X, int64_t n, int64_t d) {
  ARGCHK(X != nullptr, "X is NULL");
  ARGCHK(n >= 2, "need n >= 2 points");
  ARGCHK(d >= 1, "need d >= 1");
  if (n > kMaxPoints || d > kMaxDim) {
    set_err("n <= 700000 and d <= 32768 are supported%s (n or d is %lld)", "", (long long)(n > kMaxPoints ? n : d));
    throw Fail{ADAGIO_E_UNSUPPORTED};
  }
  if (round_up(n, kTile) * round_up(d, 128) >= ((int64_t)1 << 32)) {
    set_err("n x d beyond the supported range%s (n x d = %lld)", "", (long long)(n * d));
    throw Fail{ADAGIO_E_UNSUPPORTED};
  }
}

}  // namespace adg

using namespace adg;

extern "C" {

int adagio_pca(const float* X, int64_t n, int64_t d, double* lambda, double* Vt, void* stream) {
  return guarded([&] {
    check_points(X, n, d);
    ARGCHK(lambda && Vt, "lambda or Vt is NULL");
    hipStream_t st = as_stream(stream);
    CallWs cw(as_stream(stream));
    Workspace& ws = *cw.ws;
    Points p = prep_points(ws, X, n, d, st);
    principal_axes(ws, p, st, lambda, Vt);
    HIPCHK(hipStreamSynchronize(st));
  });
}

int adagio_pca_randomized(const float* X, int64_t n, int64_t d, int32_t ell, int32_t power_iters, uint64_t seed,
                          double* lambda, double* Vt, void* stream) {
  return guarded([&] {
    check_points(X, n, d);
    ARGCHK(lambda && Vt, "lambda or Vt is NULL");
    ARGCHK(ell >= 1 && ell <= d, "ell must be in [1, d]");
    ARGCHK(power_iters >= 0 && power_iters <= 64, "power_iters must be in [0, 64]");
    hipStream_t st = as_stream(stream);
    CallWs cw(as_stream(stream));
    Workspace& ws = *cw.ws;
    Points p = prep_points(ws, X, n, d, st);
    const int m = (int)round_up(d, 2 * bj_block());
    const double* C = full_covariance(ws, p, m, st);
    randomized_axes(ws, C, m, d, ell, power_iters, seed, lambda, Vt, st);
    HIPCHK(hipStreamSynchronize(st));
  });
}

int adagio_project_axes(const double* Vt, int64_t d, int32_t r, uint64_t seed, float* Pi_out, void* stream) {
  return guarded([&] {
    ARGCHK(Vt && Pi_out, "Vt or Pi_out is NULL");
    ARGCHK(d >= 1, "need d >= 1");
    ARGCHK(r >= 1 && r <= d, "r must be in [1, d]");
    CallWs cw(as_stream(stream));
    Workspace& ws = *cw.ws;
    build_map(ws, Vt, d, r, seed, Pi_out, as_stream(stream));
  });
}

int adagio_project_family(const double* Vt, int64_t d, int32_t r, int32_t family, uint64_t seed, float* Pi_out,
                          void* stream) {
  return guarded([&] {
    ARGCHK(Vt && Pi_out, "Vt or Pi_out is NULL");
    ARGCHK(d >= 1, "need d >= 1");
    ARGCHK(r >= 1 && r <= d, "r must be in [1, d]");
    ARGCHK(family == ADAGIO_MAP_ADAGIO || family == ADAGIO_MAP_PCA || family == ADAGIO_MAP_JL, "unknown map family");
    CallWs cw(as_stream(stream));
    Workspace& ws = *cw.ws;
    build_family_map(ws, family, Vt, d, r, seed, Pi_out, as_stream(stream));
  });
}

int adagio_project(const float* X, int64_t n, int64_t d, int32_t r, uint64_t seed, float* Pi_out, void* stream) {
  return guarded([&] {
    check_points(X, n, d);
    ARGCHK(Pi_out, "Pi_out is NULL");
    ARGCHK(r >= 1 && r <= d, "r must be in [1, d]");
    hipStream_t st = as_stream(stream);
    CallWs cw(as_stream(stream));
    Workspace& ws = *cw.ws;
    Points p = prep_points(ws, X, n, d, st);
    Axes ax = principal_axes(ws, p, st);
    build_map(ws, ax.Vt, d, r, seed, Pi_out, st);
    HIPCHK(hipStreamSynchronize(st));
  });
}

int adagio_embed(const float* X, int64_t n, int64_t d, const float* Pi, int32_t r, float* Y_out, void* stream) {
  return guarded([&] {
    ARGCHK(X && Pi && Y_out, "NULL pointer");
    ARGCHK(n >= 1 && d >= 1, "need n >= 1 and d >= 1");
    ARGCHK(r >= 1, "need r >= 1");
    (void)checked_device();
    HIPCHK(launch_embed_f32(X, n, d, Pi, r, Y_out, as_stream(stream)));
  });
}

int adagio_max_distortion(const float* X, int64_t n, int64_t d, const float* Y, int32_t r, const adagio_opts_t* opts,
                          adagio_cert_t* cert_out, void* stream) {
  return guarded([&] {
    check_points(X, n, d);
    ARGCHK(Y && cert_out, "Y or cert_out is NULL");
    ARGCHK(r >= 1, "need r >= 1");
    const int screen = opts ? opts->screen : ADAGIO_SCREEN_F32;
    ARGCHK(screen == ADAGIO_SCREEN_F32 || screen == ADAGIO_SCREEN_BF16X3 || screen == ADAGIO_SCREEN_FP8,
           "unknown screen precision");
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = as_stream(stream);
    CallWs cw(as_stream(stream));
    Workspace& ws = *cw.ws;
    Points p = prep_points(ws, X, n, d, st, screen);
    Images im = images_given(ws, p, Y, r, st);
    CertTimes tm;
    *cert_out = certificate(ws, p, im, opts ? (uint32_t)std::max(0, opts->max_candidates) : 0u, st, &tm, screen);
    if (opts && opts->stats)
      fill_stats(opts->stats, tm, 1,
                 std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
  });
}

int adagio_max_distortion_noalloc(const float* X, int64_t n, int64_t d, const float* Y, int32_t r,
                                  const adagio_opts_t* opts, adagio_cert_t* cert_out, void* stream) {
  return guarded([&] {
    check_points(X, n, d);
    ARGCHK(Y && cert_out, "Y or cert_out is NULL");
    ARGCHK(r >= 1, "need r >= 1");
    const int screen = opts ? opts->screen : ADAGIO_SCREEN_F32;
    ARGCHK(screen == ADAGIO_SCREEN_F32 || screen == ADAGIO_SCREEN_BF16X3 || screen == ADAGIO_SCREEN_FP8,
           "unknown screen precision");
    if (screen != ADAGIO_SCREEN_F32) {
      set_err("the no-allocation certificate runs the FP32 screen only%s%lld", "", 0);
      throw Fail{ADAGIO_E_UNSUPPORTED};
    }
    const size_t fixed = noalloc_fixed_bytes(n, d, r);
    const size_t cand_bytes = sizeof(int2) + sizeof(PairVal);
    if (fixed + 512 + (size_t)kScratchMinCand * cand_bytes > kScratchBytes) {
      set_err("n, d and r need %s%lld bytes of scratch; the no-allocation entry point has 64 MiB", "",
              (long long)(fixed + 512 + (size_t)kScratchMinCand * cand_bytes));
      throw Fail{ADAGIO_E_UNSUPPORTED};
    }
    uint32_t cap = (uint32_t)std::min<size_t>(kDefaultCap, (kScratchBytes - fixed - 512) / cand_bytes);
    if (opts && opts->max_candidates > 0) cap = std::min<uint32_t>(cap, (uint32_t)opts->max_candidates);
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = as_stream(stream);
    const int dev = checked_device();
    Arena arena;
    arena.base = static_cast<unsigned char*>(scratch_ptr(dev));
    arena.size = kScratchBytes;
    struct ArenaScope {
      explicit ArenaScope(Arena* a) { g_arena = a; }
      ~ArenaScope() { g_arena = nullptr; }
    } arena_scope(&arena);
    Workspace ws;   // every buffer carved from the arena; no streams or events
    Points p = prep_points(ws, X, n, d, st, screen);
    Images im = images_given(ws, p, Y, r, st);
    CertTimes tm;
    const bool timed = opts && opts->stats;
    *cert_out = certificate(ws, p, im, cap, st, timed ? &tm : nullptr, screen, nullptr, 0, -1.0, nullptr, false);
    if (timed)
      fill_stats(opts->stats, tm, 1,
                 std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
  });
}

int adagio_certify_map(const float* X, int64_t n, int64_t d, const float* Pi, int32_t r, const adagio_opts_t* opts,
                       adagio_cert_t* cert_out, void* stream) {
  return guarded([&] {
    check_points(X, n, d);
    ARGCHK(Pi && cert_out, "Pi or cert_out is NULL");
    ARGCHK(r >= 1, "need r >= 1");
    const int screen = opts ? opts->screen : ADAGIO_SCREEN_F32;
    ARGCHK(screen == ADAGIO_SCREEN_F32 || screen == ADAGIO_SCREEN_BF16X3 || screen == ADAGIO_SCREEN_FP8,
           "unknown screen precision");
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = as_stream(stream);
    CallWs cw(as_stream(stream));
    Workspace& ws = *cw.ws;
    Points p = prep_points(ws, X, n, d, st, screen);
    Images im = images_of_map(ws, p, Pi, r, st);
    CertTimes tm;
    *cert_out = certificate(ws, p, im, opts ? (uint32_t)std::max(0, opts->max_candidates) : 0u, st, &tm, screen);
    if (opts && opts->stats)
      fill_stats(opts->stats, tm, 1,
                 std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
  });
}

int adagio_fit(const float* X, int64_t n, int64_t d, double eps, uint64_t seed, const adagio_opts_t* opts,
               float* Pi_out, int32_t* r_out, int32_t* s_out, adagio_cert_t* cert_out, void* stream) {
  return guarded([&] {
    check_points(X, n, d);
    ARGCHK(Pi_out && r_out && s_out && cert_out, "NULL output pointer");
    ARGCHK(eps > 0.0 && eps < 1.0, "eps must be in (0, 1)");
    const int screen = opts ? opts->screen : ADAGIO_SCREEN_F32;
    ARGCHK(screen == ADAGIO_SCREEN_F32 || screen == ADAGIO_SCREEN_BF16X3 || screen == ADAGIO_SCREEN_FP8,
           "unknown screen precision");
    const int search = opts ? opts->search : ADAGIO_SEARCH_BISECT;
    ARGCHK(search == ADAGIO_SEARCH_BISECT || search == ADAGIO_SEARCH_LEARNED, "unknown search");
    ARGCHK(search != ADAGIO_SEARCH_LEARNED || opts->predictor, "learned search needs opts->predictor");
    const int pca = opts ? opts->pca : ADAGIO_PCA_EXACT;
    const int pca_iters = opts ? opts->pca_iters : 0;
    ARGCHK(pca == ADAGIO_PCA_EXACT || pca == ADAGIO_PCA_RANDOMIZED, "unknown PCA mode");
    ARGCHK(pca_iters >= 0 && pca_iters <= 64, "pca_iters must be in [0, 64]");
    const int family = opts ? opts->family : ADAGIO_MAP_ADAGIO;
    ARGCHK(family == ADAGIO_MAP_ADAGIO || family == ADAGIO_MAP_PCA || family == ADAGIO_MAP_JL, "unknown map family");
    ARGCHK(family == ADAGIO_MAP_ADAGIO || search == ADAGIO_SEARCH_BISECT,
           "the learned search is for Algorithm 1's maps only");
    const int no_witness = opts ? opts->no_witness : 0;
    ARGCHK(no_witness == 0 || no_witness == 1, "no_witness must be 0 or 1");
    const int refine = opts ? opts->refine : 0;
    ARGCHK(refine == 0 || refine == 1 || refine == 2, "refine must be 0, 1 or 2");
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = as_stream(stream);
    CallWs cw(as_stream(stream));
    Workspace& ws = *cw.ws;
    const uint32_t cap0 = opts ? (uint32_t)std::max(0, opts->max_candidates) : 0u;
    EvPair e_pca, e_search;
    e_pca.begin(st);
    Points p = prep_points(ws, X, n, d, st, screen);
    // The search's screens share a point-Gram cache (when it fits), filled on
    // the second stream while the PCA runs.
    float* gcache = gram_cache(ws, p);
    p.xgram_split = gcache && screen == ADAGIO_SCREEN_FP8;
    if (gcache && (screen == ADAGIO_SCREEN_BF16X3 || screen == ADAGIO_SCREEN_FP8))
      p.dscale = ensure<float>(ws.dscale, 1);
    // The fill runs beside the exact PCA while the eigensolver leaves most of
    // the GPU idle.  Past kFillBesideMaxM its per-round update (m^2 / 2048
    // workgroups, bound by HBM) fills the GPU by itself and the fill beside it
    // only time-slices with it, so the fill follows the PCA there.
    const bool exact_pca = gcache && family != ADAGIO_MAP_JL && pca == ADAGIO_PCA_EXACT;
    const bool gwait_pca = exact_pca && round_up(p.dx, 2 * bj_block()) <= kFillBesideMaxM;
    bool gwait = gcache != nullptr;
    // without the exact PCA to run beside, the fill starts at once
    if (gcache && !exact_pca) gram_fill_async(ws, p, screen, gcache, st);
    Axes ax;                         // the JL-only family needs no PCA
    const bool randomized = pca == ADAGIO_PCA_RANDOMIZED && family != ADAGIO_MAP_JL;
    const int mc = (int)round_up(d, 2 * bj_block());
    const double* Cov = nullptr;
    if (randomized) {
      Cov = full_covariance(ws, p, mc, st);
      ax.lam = ensure<double>(ws.lam, (size_t)d);
      ax.Vt = ensure<double>(ws.Vt, (size_t)(d * d));
    } else if (family != ADAGIO_MAP_JL) {
      if (gwait_pca) {
        // beside the fill: on the non-blocking third stream after the
        // centred copies, the fill starting once the covariance (a large
        // GEMM) is done, so that it runs beside the eigensolver's
        // small kernels only; st continues after the PCA
        ensure_streams(ws);
        HIPCHK(hipEventRecord(ws.ev_in, st));
        HIPCHK(hipStreamWaitEvent(ws.aux2, ws.ev_in, 0));
        ax = principal_axes(ws, p, ws.aux2, nullptr, nullptr,
                            [&] { gram_fill_async(ws, p, screen, gcache, ws.aux2); });
        HIPCHK(hipEventRecord(ws.ev_pca, ws.aux2));
        HIPCHK(hipStreamWaitEvent(st, ws.ev_pca, 0));
      } else {
        ax = principal_axes(ws, p, st);
        // after the PCA, on all CUs; the first probes' embeddings run beside it
        if (exact_pca) gram_fill_async(ws, p, screen, gcache, st, true);
      }
    }
    e_pca.end(st);
    // The images of the leading axes, kept across the probes (none for the
    // JL-only family, or past the memory budget).
    AxisImages axim;
    axim.cap = family == ADAGIO_MAP_PCA ? d : family == ADAGIO_MAP_ADAGIO ? d / 2 : 0;
    if (axim.cap > 0 && p.dx > 0 && (size_t)(p.n * axim.cap) * sizeof(double) <= kAxisImagesMaxBytes)
      axim.Y = ensure<double>(ws.axy, (size_t)(p.n * axim.cap));
    Images im_last;      // the images of the map at im_r, the last one embedded
    int64_t im_r = -1;
    // rows of the map at r that are axes
    auto lead_axes = [&](int64_t r) -> int64_t {
      return family == ADAGIO_MAP_PCA ? r : family == ADAGIO_MAP_JL ? 0 : (r == d ? d : r / 2);
    };
    // Randomized PCA: directions for the largest s needed so far plus 10.
    const int64_t kOversample = 10;
    int64_t ell_cur = 0;
    auto need_axes = [&](int64_t r) {
      if (!randomized) return;
      const int64_t sn = family == ADAGIO_MAP_PCA ? r : (r == d ? d : r / 2);
      if (sn == 0 || ell_cur == d || sn + kOversample <= ell_cur) return;
      ell_cur = std::min<int64_t>(d, sn + kOversample);
      randomized_axes(ws, Cov, mc, d, ell_cur, pca_iters, seed, ax.lam, ax.Vt, st);
      axim.s = 0;   // new axes: their images are not the kept ones
      im_r = -1;
    };
    e_search.begin(st);
    float* Pi = ensure<float>(ws.Pi, (size_t)(d * d));
    CertTimes tm;
    int ncert = 0;
    int64_t lo = 0, hi = d;
    bool have_hi = false;
    adagio_cert_t cert_hi;
    memset(&cert_hi, 0, sizeof(cert_hi));
    // The rigorous screen: the FP8 screen only ranks pairs, so an FP8 fit
    // makes its decisions with screened probes and then certifies with the
    // BF16 split screen.
    const int rig = screen == ADAGIO_SCREEN_FP8 ? ADAGIO_SCREEN_BF16X3 : screen;
    // One probe: the map at r under screen `scr`.  A certificate passes when
    // its exact maximum is <= eps, or (incomplete) when its proven bound over
    // all pairs is <= eps, and becomes the current answer.  A screened probe
    // passes when its re-evaluated maximum is <= eps; it fails only on a pair
    // that exceeds eps, but may pass a map that a certificate rejects.
    // The probes of the search's own screen load the point-Gram cache.
    // Witness pool: probes after the first certificate are first checked
    // against the worst pairs of the earlier certificates.
    uint32_t npool = 0;
    if (!no_witness) pool_reset(ws, st);
    auto probe = [&](int64_t r, int scr) {
      need_axes(r);
      build_family_map(ws, family, ax.Vt, d, r, seed, Pi, st);
      if (npool > 0) {
        const PairVal w = pool_witness(ws, p, Pi, r, npool, st);
        if (w.i >= 0 && w.v > eps + kWitnessMargin) {
          log_refuted(tm, r, 0, w.v, 3, 0.0);
          return false;
        }
      }
      // An FP8 fit certifies the r of its last screened probe, usually the
      // map embedded last: its images (and their screen copies) are reused.
      if (r != im_r) {
        im_last = images_of_map(ws, p, Pi, r, st, &axim, lead_axes(r));
        im_r = r;
      }
      const Images& im = im_last;
      // the search's own screens, and in an FP8 fit its BF16 split
      // certificates, load the fit's point-Gram cache
      const int gmode = gcache && (scr == screen || (screen == ADAGIO_SCREEN_FP8 && scr == ADAGIO_SCREEN_BF16X3)) ? 2 : 0;
      if (gmode == 2 && gwait) {
        HIPCHK(hipStreamWaitEvent(st, ws.ev_out, 0));
        gwait = false;
      }
      // Early stop on a pair certain to exceed eps
      StopOut so;
      adagio_cert_t c = certificate(ws, p, im, cap0, st, &tm, scr, gmode ? gcache : nullptr, gmode,
                                    no_witness ? -1.0 : eps, &so);
      if (so.stopped) return false;
      ++ncert;
      if (!no_witness) npool = pool_add(ws, p, st);
      if (scr == ADAGIO_SCREEN_FP8) return c.max_distortion <= eps;
      const bool pass = c.certified ? c.max_distortion <= eps : c.bound_rest <= eps;
      if (pass) {
        have_hi = true;
        cert_hi = c;
        HIPCHK(hipMemcpyAsync(Pi_out, Pi, sizeof(float) * r * d, hipMemcpyDeviceToDevice, st));
      }
      return pass;
    };
    // rel > 0: stop once the bracket (lo fails, hi passes) is within hi / rel
    auto bisect = [&](int scr, int64_t rel = 0) {
      while (hi - lo > 1 && (rel == 0 || (hi - lo) * rel > hi)) {
        const int64_t mid = (lo + hi) / 2;
        if (probe(mid, scr)) hi = mid;
        else lo = mid;
      }
    };
    int32_t r_pred = 0, fallback = 0;
    if (search == ADAGIO_SEARCH_LEARNED) {
      // The network's r is certified like any probe; if it fails, bisection
      // continues on (r_pred, d].
      float* feat = ensure<float>(ws.skfeat, 80);
      sketch_features(ws, p, eps, seed, feat, st);
      const double y = (double)mlp_predict(ws, opts->predictor, feat, st);
      int64_t rp = (int64_t)std::ceil((double)d * std::exp(std::min(y, 0.0)));
      if (rp < 1) rp = 1;
      if (rp > d) rp = d;
      r_pred = (int32_t)rp;
      if (rp < d) {
        if (probe(rp, rig)) hi = rp;
        else { lo = rp; fallback = 1; }
      }
      if (!fallback && refine) {
        // downward from the certified prediction: r / 1.25 while probes pass
        // (a failing probe is usually refuted by the witness pool the first
        // certificate filled), then bisection between the last failure and
        // the last pass: to the end (refine 1), or until the bracket is
        // within 4% of the last pass (refine 2)
        for (;;) {
          const int64_t g = (int64_t)std::floor((double)hi / 1.25);
          if (g <= lo) break;
          if (probe(g, rig)) hi = g;
          else { lo = g; break; }
        }
      }
      if (fallback) bisect(rig);
      else if (refine) bisect(rig, refine == 2 ? 25 : 0);
    } else if (screen == ADAGIO_SCREEN_FP8) {
      // Bisection over r on screened probes, then the certificate of the
      // result; if it fails, certified bisection continues on (r, d].
      bisect(ADAGIO_SCREEN_FP8);
      if (hi < d && !probe(hi, rig)) {
        lo = hi;
        hi = d;
        bisect(rig);
      }
    } else {
      // Bisection over r: lo = 0 (empty map, distortion 1), hi = d (isometry).
      bisect(rig);
    }
    if (!have_hi) {  // hi == d: no reduction (the full eigenbasis, or the identity)
      need_axes(d);
      build_family_map(ws, family, ax.Vt, d, d, seed, Pi_out, st);
      Images im = images_of_map(ws, p, Pi_out, d, st, &axim, lead_axes(d));
      cert_hi = certificate(ws, p, im, cap0, st, &tm, rig);
      ++ncert;
    }
    if (gwait) HIPCHK(hipStreamWaitEvent(st, ws.ev_out, 0));   // no probe loaded the cache
    e_search.end(st);
    HIPCHK(hipStreamSynchronize(st));
    *r_out = (int32_t)hi;
    *s_out = family == ADAGIO_MAP_PCA ? (int32_t)hi
             : family == ADAGIO_MAP_JL ? 0
             : (int32_t)(hi == d ? d : hi / 2);
    *cert_out = cert_hi;
    if (opts && opts->stats) {
      adagio_stats_t* s = opts->stats;
      fill_stats(s, tm, ncert,
                 std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
      s->t_pca_ms = e_pca.ms();
      s->t_search_ms = e_search.ms();
      s->eig_sweeps = ax.sweeps;
      s->r_predicted = r_pred;
      s->n_fallback = fallback;
      float gms = 0.0f;
      if (gcache) HIPCHK(hipEventElapsedTime(&gms, ws.ev_t0, ws.ev_t1));
      s->t_gram_ms = gms;
    }
  });
}

int adagio_quantize_fp8(const float* A, int64_t n, int64_t m, uint8_t* Q_out, float* scale_out, double* norm2_out,
                        void* stream) {
  return guarded([&] {
    ARGCHK(A && Q_out && scale_out && norm2_out, "NULL pointer");
    ARGCHK(n >= 1 && m >= 1, "need n >= 1 and m >= 1");
    (void)checked_device();
    HIPCHK(launch_quant_fp8(A, n, m, m, m, Q_out, scale_out, norm2_out, as_stream(stream)));
  });
}

int adagio_sketch_features(const float* X, int64_t n, int64_t d, double eps, uint64_t seed, float* feat_out,
                           void* stream) {
  return guarded([&] {
    check_points(X, n, d);
    ARGCHK(feat_out, "feat_out is NULL");
    ARGCHK(eps > 0.0 && eps < 1.0, "eps must be in (0, 1)");
    hipStream_t st = as_stream(stream);
    CallWs cw(as_stream(stream));
    Workspace& ws = *cw.ws;
    Points p = prep_points(ws, X, n, d, st);
    sketch_features(ws, p, eps, seed, feat_out, st);
    HIPCHK(hipStreamSynchronize(st));
  });
}

int64_t adagio_mlp_param_count(void) { return mlp_layout().total; }

int adagio_mlp_forward(const float* params, const float* feats, int32_t B, float* out, void* stream) {
  return guarded([&] {
    ARGCHK(params && feats && out, "NULL pointer");
    ARGCHK(B >= 1 && B <= (1 << 20), "batch must be in [1, 2^20]");
    hipStream_t st = as_stream(stream);
    CallWs cw(as_stream(stream));
    Workspace& ws = *cw.ws;
    const MlpLayout L = mlp_layout();
    MlpBufs b = mlp_bufs(ws, L, B);
    HIPCHK(mlp_to_bf16(params, b.pb, L.total, st));
    HIPCHK(mlp_to_bf16(feats, b.X, (int64_t)B * L.in_pad, st));
    HIPCHK(mlp_forward(L, params, b.pb, b.X, B, b.a, out, st));
  });
}

int adagio_mlp_grad(const float* params, const float* feats, const float* targets, int32_t B, float tau, float* grad,
                    float* loss, void* stream) {
  return guarded([&] {
    ARGCHK(params && feats && targets && grad && loss, "NULL pointer");
    ARGCHK(B >= 1 && B <= (1 << 20), "batch must be in [1, 2^20]");
    ARGCHK(tau > 0.0f && tau < 1.0f, "tau must be in (0, 1)");
    hipStream_t st = as_stream(stream);
    CallWs cw(as_stream(stream));
    Workspace& ws = *cw.ws;
    const MlpLayout L = mlp_layout();
    MlpBufs b = mlp_bufs(ws, L, B);
    HIPCHK(mlp_to_bf16(params, b.pb, L.total, st));
    HIPCHK(mlp_to_bf16(feats, b.X, (int64_t)B * L.in_pad, st));
    HIPCHK(hipMemsetAsync(grad, 0, sizeof(float) * L.total, st));
    HIPCHK(mlp_forward(L, params, b.pb, b.X, B, b.a, b.out, st));
    HIPCHK(mlp_backward(L, b.pb, b.X, targets, B, tau, b.a, b.out, grad, loss, st));
  });
}

int adagio_mlp_train_step(float* params, float* adam_m, float* adam_v, int32_t step, float lr, const float* feats,
                          const float* targets, int32_t B, float tau, float* loss, void* stream) {
  return guarded([&] {
    ARGCHK(params && adam_m && adam_v && feats && targets && loss, "NULL pointer");
    ARGCHK(B >= 1 && B <= (1 << 20), "batch must be in [1, 2^20]");
    ARGCHK(step >= 1, "step is 1-based");
    ARGCHK(tau > 0.0f && tau < 1.0f, "tau must be in (0, 1)");
    hipStream_t st = as_stream(stream);
    CallWs cw(as_stream(stream));
    Workspace& ws = *cw.ws;
    const MlpLayout L = mlp_layout();
    MlpBufs b = mlp_bufs(ws, L, B);
    float* grad = ensure<float>(ws.mlp_grad, (size_t)L.total);
    HIPCHK(mlp_to_bf16(params, b.pb, L.total, st));
    HIPCHK(mlp_to_bf16(feats, b.X, (int64_t)B * L.in_pad, st));
    HIPCHK(hipMemsetAsync(grad, 0, sizeof(float) * L.total, st));
    HIPCHK(mlp_forward(L, params, b.pb, b.X, B, b.a, b.out, st));
    HIPCHK(mlp_backward(L, b.pb, b.X, targets, B, tau, b.a, b.out, grad, loss, st));
    HIPCHK(mlp_adam(params, b.pb, grad, adam_m, adam_v, L.total, lr, step, st));
  });
}

int adagio_knn(const float* Q, int64_t nq, const float* D, int64_t nd, int64_t m, int32_t k, int32_t exclude_self,
               int32_t* idx_out, double* dist_out, adagio_knn_stats_t* stats_out, void* stream) {
  return guarded([&] {
    auto t0 = std::chrono::steady_clock::now();
    ARGCHK(Q && D && idx_out && dist_out, "NULL pointer");
    ARGCHK(nq >= 1 && nd >= 1 && m >= 1, "need nq, nd, m >= 1");
    ARGCHK(nd <= ((int64_t)1 << 31) - 2 && nq <= ((int64_t)1 << 31) - 2, "nq and nd must be below 2^31 - 1");
    ARGCHK(m <= ((int64_t)1 << 20), "m must be at most 2^20");
    ARGCHK(k >= 1 && k <= kKnnKeep, "k must be in [1, 32]");
    ARGCHK(exclude_self == 0 || exclude_self == 1, "exclude_self must be 0 or 1");
    ARGCHK(!exclude_self || nq <= nd, "exclude_self needs nq <= nd (query i is database row i)");
    ARGCHK(k <= nd - exclude_self, "k exceeds the number of database rows");
    hipStream_t st = as_stream(stream);
    CallWs cw(as_stream(stream));
    Workspace& ws = *cw.ws;
    const int64_t K = round_up(m, kChunk);
    const int64_t nq_pad = round_up(nq, kTile), nd_pad = round_up(nd, kTile);
    KnnView v;
    float* Qp = ensure<float>(ws.knQ, (size_t)(nq_pad * K));
    float* Dp = ensure<float>(ws.knD, (size_t)(nd_pad * K));
    double* nq64 = ensure<double>(ws.knNq64, (size_t)nq_pad);
    double* nd64 = ensure<double>(ws.knNd64, (size_t)nd_pad);
    float* nq32 = ensure<float>(ws.knNq32, (size_t)nq_pad);
    float* nd32 = ensure<float>(ws.knNd32, (size_t)nd_pad);
    double* ndmax = ensure<double>(ws.knMax, 1);
    int* cnt = ensure<int>(ws.knCnt, 2);   // [0] non-finite flag, [1] listed queries
    int* fb = ensure<int>(ws.knFb, (size_t)nq);
    EvPair e_prep, e_screen, e_finish, e_fb;
    e_prep.begin(st);
    HIPCHK(hipMemsetAsync(cnt, 0, 2 * sizeof(int), st));
    HIPCHK(launch_knn_prep(Q, nq, m, nq_pad, K, Qp, nq64, nq32, cnt, st));
    HIPCHK(launch_knn_prep(D, nd, m, nd_pad, K, Dp, nd64, nd32, cnt, st));
    HIPCHK(launch_knn_max(nd64, nd, ndmax, st));
    e_prep.end(st);
    int flags[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(flags, cnt, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (flags[0]) {
      set_err("input contains NaN or Inf%s%lld", "", 0);
      throw Fail{ADAGIO_E_NONFINITE};
    }
    v.Qp = Qp; v.Dp = Dp; v.K = K; v.m = m; v.nq32 = nq32; v.nd32 = nd32; v.nq = nq; v.nd = nd;
    v.QB = (int)(nq_pad / kKnnQueries);
    v.NTd = (int)(nd_pad / kTile);
    v.excl = exclude_self;
    // Splits of the database: enough workgroups to fill the chip several
    // times over, at most kKnnMaxSplits, every split non-empty.
    int S = (int)std::min<int64_t>({(int64_t)kKnnMaxSplits, (int64_t)v.NTd, std::max<int64_t>(1, (4096 + v.QB - 1) / v.QB)});
    v.tps = (v.NTd + S - 1) / S;
    v.S = (v.NTd + v.tps - 1) / v.tps;
    uint64_t* keys = ensure<uint64_t>(ws.knKeys, (size_t)nq_pad * v.S * kKnnKeep);
    // shared per-query thresholds, order-preserving bits of +inf to start
    unsigned* tau_g = ensure<unsigned>(ws.knTau, (size_t)nq_pad);
    e_screen.begin(st);
    HIPCHK(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(tau_g), 0xFF800000, (size_t)nq_pad, st));
    HIPCHK(launch_knn_screen(v, keys, tau_g, st));
    e_screen.end(st);
    // |est - d| <= c_K (N_q + N_x): the screen constant of an FP32 Gram of K terms;
    // the FP64 sums of m squares are within (m + 4) u64 (relative) of d.
    const double cK = ((double)K + 32.0) * kU32 * 1.001;
    const double g64 = ((double)m + 4.0) * kU64 * 1.01;
    e_finish.begin(st);
    HIPCHK(launch_knn_finish(v, keys, Q, D, nq64, ndmax, tau_g, cK, g64, k, idx_out, dist_out, cnt + 1, fb, st));
    e_finish.end(st);
    HIPCHK(hipMemcpyAsync(flags + 1, cnt + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int nfb = flags[1];
    double t_fb = 0.0;
    if (nfb > 0) {
      e_fb.begin(st);
      HIPCHK(launch_knn_fallback(Q, D, m, nd, k, exclude_self, fb, nfb, idx_out, dist_out, st));
      e_fb.end(st);
      HIPCHK(hipStreamSynchronize(st));
      t_fb = e_fb.ms();
    }
    if (stats_out) {
      adagio_knn_stats_t o;
      memset(&o, 0, sizeof(o));
      o.splits = v.S;
      o.n_fallback = nfb;
      o.t_prep_ms = e_prep.ms();
      o.t_screen_ms = e_screen.ms();
      o.t_finish_ms = e_finish.ms();
      o.t_fallback_ms = t_fb;
      o.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      *stats_out = o;
    }
  });
}

int adagio_knn_vote(const int32_t* nn_idx, int64_t nq, int32_t k, const int32_t* d_label, int64_t nd,
                    int32_t n_labels, int32_t group, int32_t* label_out, void* stream) {
  return guarded([&] {
    ARGCHK(nn_idx && d_label && label_out, "NULL pointer");
    ARGCHK(nq >= 1 && nd >= 1 && k >= 1, "need nq, nd, k >= 1");
    ARGCHK(n_labels >= 1 && n_labels <= 8192, "n_labels must be in [1, 8192]");
    ARGCHK(group >= 1, "group must be >= 1");
    hipStream_t st = as_stream(stream);
    CallWs cw(as_stream(stream));
    Workspace& ws = *cw.ws;
    int* bad = ensure<int>(ws.knCnt, 2);
    HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), st));
    HIPCHK(launch_knn_vote(nn_idx, nq, k, d_label, nd, n_labels, group, label_out, bad, st));
    int h = 0;
    HIPCHK(hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    ARGCHK(!h, "a neighbour index or label is out of range");
  });
}

int adagio_mfma_ceiling(int32_t kind, double* tflops_out, double* ghz_out, void* stream) {
  return guarded([&] {
    ARGCHK(kind >= 0 && kind <= 2, "kind must be 0 (FP8), 1 (BF16) or 2 (FP32)");
    ARGCHK(tflops_out && ghz_out, "NULL output pointer");
    hipStream_t st = as_stream(stream);
    // operands: 1024 words of e4m3 byte patterns without NaN codes (FP8);
    // the BF16 and FP32 loops read values from the same words
    std::vector<int> h(1024);
    uint32_t z = 0x9E3779B9u;
    for (int& x : h) {
      uint32_t w = 0;
      for (int k = 0; k < 4; ++k) {
        z = z * 1664525u + 1013904223u;
        uint32_t b = (z >> 24) & 0xFFu;
        if ((b & 0x7Fu) == 0x7Fu) b = 0x38u;
        w |= b << (8 * k);
      }
      x = (int)w;
    }
    DevBuf bin, bout, bclk;
    int* din = ensure<int>(bin, 1024);
    float* dout = ensure<float>(bout, (size_t)mfma_ceiling_grid() * 256);
    unsigned long long* dclk = ensure<unsigned long long>(bclk, 2);
    HIPCHK(hipMemcpyAsync(din, h.data(), 4096, hipMemcpyHostToDevice, st));
    // about 2.5 ms per launch; the last of four is timed, after the clock
    // has settled under the load
    const int iters = kind == 0 ? 4096 : kind == 1 ? 8192 : 2048;
    const double flop = (kind == 0 ? 32.0 * 32 * 64 : kind == 1 ? 32.0 * 32 * 16 : 32.0 * 32 * 2) * 2.0 * 4.0 *
                        iters * mfma_ceiling_grid() * 4.0;
    struct Ev {
      hipEvent_t e = nullptr;
      ~Ev() { if (e) (void)hipEventDestroy(e); }
    } e0, e1;
    HIPCHK(hipEventCreate(&e0.e));
    HIPCHK(hipEventCreate(&e1.e));
    for (int rep = 0; rep < 3; ++rep) HIPCHK(launch_mfma_ceiling(kind, din, dout, dclk, iters, st));
    HIPCHK(hipEventRecord(e0.e, st));
    HIPCHK(launch_mfma_ceiling(kind, din, dout, dclk, iters, st));
    HIPCHK(hipEventRecord(e1.e, st));
    unsigned long long c[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(c, dclk, sizeof(c), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, e0.e, e1.e));
    *tflops_out = ms > 0.0f ? flop / ((double)ms * 1e9) : 0.0;
    *ghz_out = c[1] ? (double)c[0] / ((double)c[1] / 100e6) / 1e9 : 0.0;
  });
}

int adagio_release(void) {
  return guarded([&] {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64 || !g_kept[dev]) return;
    delete g_kept[dev];
    g_kept[dev] = nullptr;
  });
}

int adagio_keep_workspace(int keep) {
  return guarded([&] {
    ARGCHK(keep == 0 || keep == 1, "keep must be 0 or 1");
    g_keep = keep == 1;
    if (!g_keep) release_kept_all();
  });
}

const char* adagio_status_string(int status) {
  switch (status) {
    case ADAGIO_OK: return "ok";
    case ADAGIO_E_INVALID_ARG: return "invalid argument";
    case ADAGIO_E_NONFINITE: return "non-finite input";
    case ADAGIO_E_HIP: return "HIP runtime error";
    case ADAGIO_E_OOM: return "out of device memory";
    case ADAGIO_E_UNSUPPORTED: return "unsupported device or size";
    case ADAGIO_E_NO_CONVERGENCE: return "eigensolver did not converge";
    case ADAGIO_E_CAPACITY: return "candidate capacity exceeded";
    case ADAGIO_E_NOT_CERTIFIED: return "certificate incomplete";
    default: return "unknown status";
  }
}

const char* adagio_last_error(void) { return g_err.c_str(); }

}  // extern "C"
