"""Algorithm 1's linear map (oracle, FP64).  Test infrastructure only.

Paper: Algorithm 1 maps each point w to (P w, S (w - P^T P w)), where P (s x d)
has orthonormal rows and S (k x d) is the +-1/sqrt(k) JL matrix; the proof of
Theorem 2 writes Q = I - P^T P, so the map is the (s + k) x d matrix
Pi = [P ; S Q].  Sec. 4.1 "Implementation": for a target dimension r the paper
uses floor(r/2) principal components and ceil(r/2) JL rows.

Readings:
* r = d means "no reduction" (Table 3's JL rows, Sec. 4.4): Pi = V^T, the full
  orthonormal eigenbasis, which is an isometry.  The printed floor/ceil split
  at r = d would not be one.
* The map is linear and is not shifted by the mean (f(w) = Pi w as printed);
  distances do not depend on a shift.
* S Q is formed as S - (S P^T) P, which equals S (I - P^T P) exactly in real
  arithmetic without building the d x d projector.
"""
import numpy as np

from .jl_signs import jl_matrix


def split(r, d):
    """(s, k) for target dimension r: floor(r/2) PCA rows, ceil(r/2) JL rows;
    r = d gives (d, 0)."""
    if not 1 <= r <= d:
        raise ValueError("r must be in [1, d]")
    if r == d:
        return d, 0
    return r // 2, r - r // 2


def adagio_map(Vt, r, seed):
    """Pi_r = [P ; S Q] (r x d, FP64) from sorted eigenvectors Vt (rows)."""
    d = Vt.shape[1]
    s, k = split(r, d)
    P = Vt[:s]
    if k == 0:
        return P.copy()
    S = jl_matrix(seed, k, d)
    SQ = S - (S @ P.T) @ P
    return np.vstack([P, SQ])


def pca_map(Vt, r):
    """PCA alone: the top-r principal directions (Table 3's PCA rows)."""
    return Vt[:r].copy()


def jl_map(d, r, seed):
    """JL alone: Lemma 1's r x d +-1/sqrt(r) matrix (Table 3's JL rows);
    r = d means no reduction (identity)."""
    if r == d:
        return np.eye(d)
    return jl_matrix(seed, r, d)


def family_map(family, Vt, r, seed):
    """Pi_r of one of the three map families compared in Table 3 (Sec. 4.4)."""
    if family == "adagio":
        return adagio_map(Vt, r, seed)
    if family == "pca":
        return pca_map(Vt, r)
    if family == "jl":
        return jl_map(Vt.shape[1], r, seed)
    raise ValueError(family)


def embed(X, Pi):
    """f(w) = Pi w for every row w of X (FP64)."""
    return np.asarray(X, dtype=np.float64) @ np.asarray(Pi, dtype=np.float64).T
