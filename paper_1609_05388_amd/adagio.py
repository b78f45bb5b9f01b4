"""Python binding of libadagio.so (argument marshalling only).

Every function takes and returns torch tensors on the current ROCm device and
passes their device pointers and torch's current HIP stream to the C ABI of
include/adagio.h.  No computation happens here: if the shared library is
missing, ``load()`` raises instead of falling back to anything else.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadagio.so")

SCREEN = {"f32": 0, "bf16x3": 1, "fp8": 2}
SEARCH = {"bisect": 0, "learned": 1}
FAMILY = {"adagio": 0, "pca": 1, "jl": 2}
PCA = {"exact": 0, "randomized": 1}


class AdagioError(RuntimeError):
    def __init__(self, code, text):
        super().__init__("adagio error %d: %s" % (code, text))
        self.code = code


class Cert(ctypes.Structure):
    _fields_ = [("max_distortion", ctypes.c_double), ("i", ctypes.c_int64), ("j", ctypes.c_int64),
                ("side", ctypes.c_int32), ("certified", ctypes.c_int32),
                ("runner_up", ctypes.c_double), ("i2", ctypes.c_int64), ("j2", ctypes.c_int64),
                ("bound_rest", ctypes.c_double), ("n_rescored", ctypes.c_int64),
                ("n_pairs", ctypes.c_int64), ("n_flagged_tiles", ctypes.c_int64)]

    def to_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [("t_total_ms", ctypes.c_double), ("t_pca_ms", ctypes.c_double),
                ("t_search_ms", ctypes.c_double), ("t_screen_ms", ctypes.c_double),
                ("t_rescore_ms", ctypes.c_double), ("n_certificates", ctypes.c_int32),
                ("eig_sweeps", ctypes.c_int32), ("n_fallback", ctypes.c_int32),
                ("r_predicted", ctypes.c_int32), ("n_flagged_tiles", ctypes.c_int64),
                ("n_rescored", ctypes.c_int64), ("n_probes", ctypes.c_int32),
                ("n_screened", ctypes.c_int32), ("probe_r", ctypes.c_int32 * 48),
                ("probe_delta", ctypes.c_double * 48), ("probe_screen_ms", ctypes.c_double * 48),
                ("probe_gram", ctypes.c_int32 * 48), ("n_refuted", ctypes.c_int32),
                ("t_gram_ms", ctypes.c_double), ("probe_cols", ctypes.c_int32 * 48)]

    def to_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            if name.startswith("probe_"):
                v = list(v)[:self.n_probes]
            out[name] = v
        return out


class KnnStats(ctypes.Structure):
    _fields_ = [("t_total_ms", ctypes.c_double), ("t_prep_ms", ctypes.c_double),
                ("t_screen_ms", ctypes.c_double), ("t_finish_ms", ctypes.c_double),
                ("t_fallback_ms", ctypes.c_double), ("splits", ctypes.c_int32),
                ("n_fallback", ctypes.c_int32), ("reserved", ctypes.c_int64 * 4)]

    def to_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class Opts(ctypes.Structure):
    _fields_ = [("screen", ctypes.c_int32), ("search", ctypes.c_int32),
                ("max_candidates", ctypes.c_int32), ("family", ctypes.c_int32),
                ("predictor", ctypes.c_void_p), ("stats", ctypes.POINTER(Stats)),
                ("pca", ctypes.c_int32), ("pca_iters", ctypes.c_int32), ("no_witness", ctypes.c_int32),
                ("refine", ctypes.c_int32)]


_lib = None

# name -> (restype, argtypes) of every exported entry point
_P, _I64, _I32, _U64, _D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
SIGNATURES = {
    "adagio_pca": (ctypes.c_int, [_P, _I64, _I64, _P, _P, _P]),
    "adagio_pca_randomized": (ctypes.c_int, [_P, _I64, _I64, _I32, _I32, _U64, _P, _P, _P]),
    "adagio_project_axes": (ctypes.c_int, [_P, _I64, _I32, _U64, _P, _P]),
    "adagio_project": (ctypes.c_int, [_P, _I64, _I64, _I32, _U64, _P, _P]),
    "adagio_project_family": (ctypes.c_int, [_P, _I64, _I32, _I32, _U64, _P, _P]),
    "adagio_embed": (ctypes.c_int, [_P, _I64, _I64, _P, _I32, _P, _P]),
    "adagio_max_distortion": (ctypes.c_int, [_P, _I64, _I64, _P, _I32, ctypes.POINTER(Opts),
                                             ctypes.POINTER(Cert), _P]),
    "adagio_max_distortion_noalloc": (ctypes.c_int, [_P, _I64, _I64, _P, _I32, ctypes.POINTER(Opts),
                                                     ctypes.POINTER(Cert), _P]),
    "adagio_certify_map": (ctypes.c_int, [_P, _I64, _I64, _P, _I32, ctypes.POINTER(Opts),
                                          ctypes.POINTER(Cert), _P]),
    "adagio_fit": (ctypes.c_int, [_P, _I64, _I64, _D, _U64, ctypes.POINTER(Opts), _P,
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(Cert), _P]),
    "adagio_sketch_features": (ctypes.c_int, [_P, _I64, _I64, _D, _U64, _P, _P]),
    "adagio_quantize_fp8": (ctypes.c_int, [_P, _I64, _I64, _P, _P, _P, _P]),
    "adagio_mlp_param_count": (ctypes.c_int64, []),
    "adagio_mlp_forward": (ctypes.c_int, [_P, _P, _I32, _P, _P]),
    "adagio_mlp_grad": (ctypes.c_int, [_P, _P, _P, _I32, ctypes.c_float, _P, _P, _P]),
    "adagio_mlp_train_step": (ctypes.c_int, [_P, _P, _P, _I32, ctypes.c_float, _P, _P, _I32, ctypes.c_float,
                                             _P, _P]),
    "adagio_knn": (ctypes.c_int, [_P, _I64, _P, _I64, _I64, _I32, _I32, _P, _P, ctypes.POINTER(KnnStats), _P]),
    "adagio_knn_vote": (ctypes.c_int, [_P, _I64, _I32, _P, _I64, _I32, _I32, _P, _P]),
    "adagio_release": (ctypes.c_int, []),
    "adagio_mfma_ceiling": (ctypes.c_int, [_I32, ctypes.POINTER(_D), ctypes.POINTER(_D), _P]),
    "adagio_keep_workspace": (ctypes.c_int, [ctypes.c_int]),
    "adagio_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "adagio_last_error": (ctypes.c_char_p, []),
}


def load(path=LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError("libadagio.so not built at %s; run __graft_entry__.build()" % path)
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc):
    if rc != 0:
        lib = load()
        raise AdagioError(rc, "%s: %s" % (lib.adagio_status_string(rc).decode(),
                                          lib.adagio_last_error().decode()))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a torch tensor on the GPU" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s" % (name, dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


def _opts(screen="f32", search="bisect", max_candidates=0, predictor=None, stats=None, family="adagio",
          pca="exact", pca_iters=2, witness=True, refine=False):
    o = Opts()
    o.no_witness = 0 if witness else 1
    o.refine = 2 if refine == "within4" else int(refine)
    o.screen = SCREEN[screen]
    o.search = SEARCH[search]
    o.family = FAMILY[family]
    o.pca = PCA[pca]
    o.pca_iters = int(pca_iters)
    o.max_candidates = int(max_candidates)
    o.predictor = ctypes.c_void_p(predictor.data_ptr()) if predictor is not None else None
    o.stats = ctypes.pointer(stats) if stats is not None else None
    return o


def pca(X):
    """(lambda, Vt): eigenvalues (decreasing) and eigenvectors (rows), FP64."""
    lib = load()
    n, d = X.shape
    lam = torch.empty(d, dtype=torch.float64, device=X.device)
    Vt = torch.empty((d, d), dtype=torch.float64, device=X.device)
    _check(lib.adagio_pca(_dev(X, torch.float32, "X"), n, d, _dev(lam, torch.float64, "lam"),
                          _dev(Vt, torch.float64, "Vt"), _stream()))
    return lam, Vt


def pca_randomized(X, ell, power_iters, seed):
    """(lambda, Vt): ell approximate principal values and directions (rows), FP64."""
    lib = load()
    n, d = X.shape
    lam = torch.empty(ell, dtype=torch.float64, device=X.device)
    Vt = torch.empty((ell, d), dtype=torch.float64, device=X.device)
    _check(lib.adagio_pca_randomized(_dev(X, torch.float32, "X"), n, d, int(ell), int(power_iters), int(seed),
                                     _dev(lam, torch.float64, "lambda"), _dev(Vt, torch.float64, "Vt"), _stream()))
    return lam, Vt


def project_axes(Vt, r, seed):
    lib = load()
    d = Vt.shape[1]
    Pi = torch.empty((r, d), dtype=torch.float32, device=Vt.device)
    _check(lib.adagio_project_axes(_dev(Vt, torch.float64, "Vt"), d, int(r), int(seed),
                                   _dev(Pi, torch.float32, "Pi"), _stream()))
    return Pi


def project_family(Vt, r, family, seed):
    """r x d FP32 map of a family ("adagio", "pca", "jl") from sorted axes Vt."""
    lib = load()
    d = Vt.shape[1]
    Pi = torch.empty((r, d), dtype=torch.float32, device=Vt.device)
    _check(lib.adagio_project_family(_dev(Vt, torch.float64, "Vt"), d, int(r), FAMILY[family], int(seed),
                                     _dev(Pi, torch.float32, "Pi"), _stream()))
    return Pi


def project(X, r, seed):
    lib = load()
    n, d = X.shape
    Pi = torch.empty((r, d), dtype=torch.float32, device=X.device)
    _check(lib.adagio_project(_dev(X, torch.float32, "X"), n, d, int(r), int(seed),
                              _dev(Pi, torch.float32, "Pi"), _stream()))
    return Pi


def embed(X, Pi):
    lib = load()
    n, d = X.shape
    r = Pi.shape[0]
    if Pi.shape[1] != d:
        raise ValueError("Pi must be r x d")
    Y = torch.empty((n, r), dtype=torch.float32, device=X.device)
    _check(lib.adagio_embed(_dev(X, torch.float32, "X"), n, d, _dev(Pi, torch.float32, "Pi"), r,
                            _dev(Y, torch.float32, "Y"), _stream()))
    return Y


def max_distortion(X, Y, screen="f32", max_candidates=0, with_stats=False):
    lib = load()
    n, d = X.shape
    if Y.shape[0] != n:
        raise ValueError("Y must have one row per point")
    st = Stats() if with_stats else None
    o = _opts(screen, max_candidates=max_candidates, stats=st)
    c = Cert()
    _check(lib.adagio_max_distortion(_dev(X, torch.float32, "X"), n, d, _dev(Y, torch.float32, "Y"),
                                     Y.shape[1], ctypes.byref(o), ctypes.byref(c), _stream()))
    out = c.to_dict()
    if st is not None:
        out["stats"] = st.to_dict()
    return out


def max_distortion_noalloc(X, Y, max_candidates=0, with_stats=False):
    """adagio_max_distortion_noalloc: the FP32-screen certificate with every
    buffer in the library's fixed device array (no allocation)."""
    lib = load()
    n, d = X.shape
    if Y.shape[0] != n:
        raise ValueError("Y must have one row per point")
    st = Stats() if with_stats else None
    o = _opts("f32", max_candidates=max_candidates, stats=st)
    c = Cert()
    _check(lib.adagio_max_distortion_noalloc(_dev(X, torch.float32, "X"), n, d, _dev(Y, torch.float32, "Y"),
                                             Y.shape[1], ctypes.byref(o), ctypes.byref(c), _stream()))
    out = c.to_dict()
    if st is not None:
        out["stats"] = st.to_dict()
    return out


def certify_map(X, Pi, screen="f32", max_candidates=0, with_stats=False):
    lib = load()
    n, d = X.shape
    if Pi.shape[1] != d:
        raise ValueError("Pi must be r x d")
    st = Stats() if with_stats else None
    o = _opts(screen, max_candidates=max_candidates, stats=st)
    c = Cert()
    _check(lib.adagio_certify_map(_dev(X, torch.float32, "X"), n, d, _dev(Pi, torch.float32, "Pi"),
                                  Pi.shape[0], ctypes.byref(o), ctypes.byref(c), _stream()))
    out = c.to_dict()
    if st is not None:
        out["stats"] = st.to_dict()
    return out


def fit(X, eps, seed, screen="f32", search="bisect", predictor=None, max_candidates=0, family="adagio",
        pca="exact", pca_iters=2, witness=True, refine=False):
    """Returns dict(Pi=(r x d tensor), r, s, k, cert, stats).  family: "adagio"
    (Algorithm 1), "pca" or "jl" (Table 3's single-component maps); pca:
    "exact" or "randomized" (Sec. 4.5's variant, pca_iters power iterations);
    witness=False certifies every probe in full; refine=True makes the
    learned search probe downward from a certified prediction to the
    bisection-minimal r, refine="within4" stops that downward bisection once
    its last failing r is within 4% of the returned one."""
    lib = load()
    n, d = X.shape
    Pi_buf = torch.empty((d, d), dtype=torch.float32, device=X.device)
    st = Stats()
    o = _opts(screen, search, max_candidates, predictor, st, family, pca, pca_iters, witness, refine)
    r = ctypes.c_int32()
    s = ctypes.c_int32()
    c = Cert()
    _check(lib.adagio_fit(_dev(X, torch.float32, "X"), n, d, float(eps), int(seed), ctypes.byref(o),
                          _dev(Pi_buf, torch.float32, "Pi"), ctypes.byref(r), ctypes.byref(s),
                          ctypes.byref(c), _stream()))
    rv = r.value
    return {"Pi": Pi_buf[:rv], "r": rv, "s": s.value, "k": rv - s.value if rv < d else 0,
            "cert": c.to_dict(), "stats": st.to_dict()}


N_FEATURES = 80


def quantize_fp8(A):
    """(Q, scale, norm2): per-row scaled OCP e4m3 bytes (uint8, n x m), the row
    scales (FP32) and s_i^2 |q_i|^2 (FP64) of the FP32 rows of A."""
    lib = load()
    n, m = A.shape
    Q = torch.empty((n, m), dtype=torch.uint8, device=A.device)
    scale = torch.empty(n, dtype=torch.float32, device=A.device)
    norm2 = torch.empty(n, dtype=torch.float64, device=A.device)
    _check(lib.adagio_quantize_fp8(_dev(A, torch.float32, "A"), n, m, _dev(Q, torch.uint8, "Q"),
                                   _dev(scale, torch.float32, "scale"), _dev(norm2, torch.float64, "norm2"),
                                   _stream()))
    return Q, scale, norm2


def sketch_features(X, eps, seed):
    """80 predictor inputs (device FP32) of cloud X at target eps."""
    lib = load()
    n, d = X.shape
    f = torch.empty(N_FEATURES, dtype=torch.float32, device=X.device)
    _check(lib.adagio_sketch_features(_dev(X, torch.float32, "X"), n, d, float(eps), int(seed),
                                      _dev(f, torch.float32, "feat"), _stream()))
    return f


def mlp_param_count():
    return int(load().adagio_mlp_param_count())


def mlp_forward(params, feats):
    lib = load()
    B = feats.shape[0]
    out = torch.empty(B, dtype=torch.float32, device=feats.device)
    _check(lib.adagio_mlp_forward(_dev(params, torch.float32, "params"), _dev(feats, torch.float32, "feats"), B,
                                  _dev(out, torch.float32, "out"), _stream()))
    return out


def mlp_grad(params, feats, targets, tau):
    lib = load()
    B = feats.shape[0]
    grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=params.device)
    _check(lib.adagio_mlp_grad(_dev(params, torch.float32, "params"), _dev(feats, torch.float32, "feats"),
                               _dev(targets, torch.float32, "targets"), B, float(tau),
                               _dev(grad, torch.float32, "grad"), _dev(loss, torch.float32, "loss"), _stream()))
    return grad, loss


def mlp_train_step(params, adam_m, adam_v, step, lr, feats, targets, tau):
    """One Adam step in place on params/adam_m/adam_v; returns the device loss."""
    lib = load()
    B = feats.shape[0]
    loss = torch.empty(1, dtype=torch.float32, device=params.device)
    _check(lib.adagio_mlp_train_step(_dev(params, torch.float32, "params"), _dev(adam_m, torch.float32, "m"),
                                     _dev(adam_v, torch.float32, "v"), int(step), float(lr),
                                     _dev(feats, torch.float32, "feats"), _dev(targets, torch.float32, "targets"),
                                     B, float(tau), _dev(loss, torch.float32, "loss"), _stream()))
    return loss


def knn(Q, D, k, exclude_self=False):
    """(idx, dist, stats): the k nearest rows of D (device nd x m FP32) to each
    row of Q (device nq x m FP32), int32 indices and FP64 squared distances,
    ordered by (distance, index)."""
    lib = load()
    nq, m = Q.shape
    nd, m2 = D.shape
    if m != m2:
        raise ValueError("Q and D need the same number of columns")
    idx = torch.empty((nq, k), dtype=torch.int32, device=Q.device)
    dist = torch.empty((nq, k), dtype=torch.float64, device=Q.device)
    st = KnnStats()
    _check(lib.adagio_knn(_dev(Q, torch.float32, "Q"), nq, _dev(D, torch.float32, "D"), nd, m, int(k),
                          int(bool(exclude_self)), _dev(idx, torch.int32, "idx"), _dev(dist, torch.float64, "dist"),
                          ctypes.byref(st), _stream()))
    return idx, dist, st.to_dict()


def knn_vote(nn_idx, d_label, n_labels, group):
    """Majority label per group of ``group`` consecutive queries (int32)."""
    lib = load()
    nq, k = nn_idx.shape
    out = torch.empty((nq + group - 1) // group, dtype=torch.int32, device=nn_idx.device)
    _check(lib.adagio_knn_vote(_dev(nn_idx, torch.int32, "nn_idx"), nq, k, _dev(d_label, torch.int32, "d_label"),
                               d_label.shape[0], int(n_labels), int(group), _dev(out, torch.int32, "out"),
                               _stream()))
    return out


def release():
    """Frees the current device's kept workspace."""
    _check(load().adagio_release())


MFMA_KINDS = {"fp8": 0, "bf16": 1, "fp32": 2}


def mfma_ceiling(kind):
    """Throughput (TFLOP/s) of a kernel of independent MFMAs of `kind`
    ("fp8", "bf16" or "fp32") on this device, and the shader clock (GHz) it
    ran at: the attainable matrix-core rate under a sustained load."""
    lib = load()
    t = ctypes.c_double()
    g = ctypes.c_double()
    _check(lib.adagio_mfma_ceiling(MFMA_KINDS[kind], ctypes.byref(t), ctypes.byref(g), _stream()))
    return {"tflops": t.value, "clock_ghz": g.value}


def keep_workspace(keep=True):
    """Keep one workspace per device across calls (True), or free each call's
    workspace before it returns (False, the library's default)."""
    _check(load().adagio_keep_workspace(1 if keep else 0))
