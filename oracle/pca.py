"""Centring, covariance and principal subspace (oracle, FP64).  Test
infrastructure only.

Paper: Sec. 2, PCA paragraph -- PCA minimises eq. (4) once the cloud is
zero-centred and is obtained from the SVD of the data matrix; Sec. 3, opening
paragraph -- P holds the top s singular directions of the data; Sec. 4.1
"Implementation" -- PCA is sklearn's (which centres the data).

Reading (the orientation of X is garbled between Sec. 2 and Sec. 3): with
points as rows of X (n x d), P's rows are the top-s eigenvectors of the d x d
covariance C = Xc^T Xc of the centred points Xc = X - 1 mu^T.  Those are the
top right singular vectors of Xc, i.e. the paper's "left singular vectors" when
points are columns.  Only the projector P^T P matters to any distance
(eigenvector signs and rotations inside a repeated eigenvalue are free).
"""
import numpy as np


def center(X):
    """mu = mean of the rows, Xc = X - mu (both FP64)."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0)
    return mu, X - mu


def covariance(Xc):
    """C = Xc^T Xc (unnormalised; the scale does not move eigenvectors)."""
    return Xc.T @ Xc


def principal_axes(C):
    """Eigenpairs of the symmetric C sorted by decreasing eigenvalue.

    Returns (lam, Vt): lam[i] is the i-th largest eigenvalue and Vt[i] its unit
    eigenvector (so the top-s principal matrix is P = Vt[:s]).  Equal
    eigenvalues keep LAPACK's order reversed; any order is a valid answer.
    """
    lam, V = np.linalg.eigh(C)
    order = np.argsort(-lam, kind="stable")
    return lam[order], V[:, order].T.copy()


def pca(X):
    """Steps in paper order: centre, covariance, sorted eigenpairs."""
    mu, Xc = center(X)
    C = covariance(Xc)
    lam, Vt = principal_axes(C)
    return mu, C, lam, Vt
