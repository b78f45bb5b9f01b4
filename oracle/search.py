"""Target-dimension search and the full fit (oracle, FP64).  Test
infrastructure only.

Paper: Sec. 4.3 (Fig. 6) and Sec. 4.4 (Table 3) ask, for a distortion level delta, how many
dimensions each method needs; Sec. 4.1 "Implementation" fixes the
floor(r/2)/ceil(r/2) split; Algorithm 1 gives the map.

Readings:
* The API's ``eps`` is the absolute target max distortion (Table 3's delta),
  not Algorithm 1's multiplicative reduction factor.
* The search procedure is not stated.  Bisection over r: lo = 0 (the empty map
  collapses every distance, distortion 1 by convention), hi = d (the full
  eigenbasis, distortion 0).  While hi - lo > 1: mid = (lo + hi) // 2; if the
  certified distortion of Pi_mid is <= eps then hi = mid, else lo = mid.
  Result r* = hi.  The distortion is not monotone in r (S is random and s, k
  both move), so r* satisfies the target but is only bisection-minimal.
"""
import numpy as np

from . import certificate, embedding, pca


def distortion_of_map(X, Pi):
    """eq. (3) for the linear map Pi on the rows of X."""
    return certificate.certify(X, embedding.embed(X, Pi))


def fit(X, eps, seed, principal=None, monitor=None, family="adagio"):
    """Steps in paper order: PCA once, then the r search with Algorithm 1's
    map certified by eq. (3) at each probe.  Returns a dict with Pi, r, s, k,
    the certificate of Pi and the probe log."""
    if not 0.0 < eps < 1.0:
        raise ValueError("eps must be in (0, 1)")
    X = np.asarray(X, dtype=np.float64)
    if X.shape[0] < 2 or not np.all(np.isfinite(X)):
        raise ValueError("need n >= 2 finite points")
    n, d = X.shape
    if principal is None:
        _, _, lam, Vt = pca.pca(X)
    else:
        lam, Vt = principal
    lo, hi = 0, d
    probes = []
    cert_hi = None
    while hi - lo > 1:
        mid = (lo + hi) // 2
        cert = distortion_of_map(X, embedding.family_map(family, Vt, mid, seed))
        probes.append((mid, cert["max"]))
        if monitor is not None:
            monitor(mid, cert)
        if cert["max"] <= eps:
            hi, cert_hi = mid, cert
        else:
            lo = mid
    Pi = embedding.family_map(family, Vt, hi, seed)
    if cert_hi is None:
        cert_hi = distortion_of_map(X, Pi)
    s, k = embedding.split(hi, d) if family == "adagio" else (None, None)
    return {"Pi": Pi, "r": hi, "s": s, "k": k, "cert": cert_hi, "probes": probes,
            "lam": lam, "Vt": Vt}


def fit_fixed_rank(X, r, seed):
    """Algorithm 1 at a given target dimension r (Sec. 4.2's fixed-r runs)."""
    _, _, lam, Vt = pca.pca(X)
    return embedding.adagio_map(Vt, r, seed)
