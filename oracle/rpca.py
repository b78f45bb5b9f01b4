"""Randomized PCA of Sec. 4.5's Adagio-Randomized-PCA (oracle, FP64).

Test infrastructure only: the library never imports this module.

The paper swaps the exact PCA for the randomized one of Martinsson et al.
(Halko, Martinsson & Tropp's randomized range finder with subspace
iteration): for the covariance C of the centred cloud, a block Omega of ell
random test vectors, Y = C Omega, then q more products with C, each applied
to an orthonormal basis of the previous block, and the Rayleigh-Ritz step on
the final basis Q: the eigenpairs (lambda, W) of Q^T C Q give the ell
approximate principal directions Q W.

Readings: Omega holds +-1 signs (a Rademacher test matrix) from the same
counter-based SplitMix64 scheme as the JL signs, on the stream
seed ^ 0x94D049BB133111EB (scaled by 1/sqrt(ell), which changes no span);
"q power iterations" are q products beyond the first; orthonormal bases come
from numpy's QR (any basis of the same span gives the same result).
"""
import numpy as np

from .jl_signs import jl_matrix

STREAM = 0x94D049BB133111EB


def randomized_axes(C, ell, q, seed):
    """(lambda, Vt): ell approximate eigenpairs of the symmetric C, values
    decreasing, Vt rows = unit directions."""
    C = np.asarray(C, dtype=np.float64)
    d = C.shape[0]
    if not 1 <= ell <= d:
        raise ValueError("ell must be in [1, d]")
    Omega = jl_matrix(np.uint64(seed) ^ np.uint64(STREAM), ell, d).T     # d x ell
    Q = Omega
    for _ in range(q + 1):
        Q, _ = np.linalg.qr(C @ Q)
    B = Q.T @ C @ Q
    lam, W = np.linalg.eigh((B + B.T) / 2)
    order = np.argsort(-lam, kind="stable")
    return lam[order], (Q @ W[:, order]).T


def randomized_pca(X, ell, q, seed):
    """Randomized PCA of the rows of X: covariance of the centred cloud, then
    randomized_axes."""
    X = np.asarray(X, dtype=np.float64)
    Xc = X - X.mean(axis=0)
    return randomized_axes(Xc.T @ Xc, ell, q, seed)
