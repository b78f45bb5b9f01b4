"""Pins of the oracle's randomized PCA (Sec. 4.5's variant) against what the
mathematics fixes: exact recovery of an exactly low-rank covariance, the full
block (ell = d) reproducing every eigenpair, Cauchy interlacing of the Ritz
values, independence from the orthonormalisation method, and convergence
with power iterations."""
import numpy as np

from oracle import jl_signs, rpca
from paper_1609_05388_amd import gen


def angles_cos(A, B):
    """Cosines of the principal angles between the row spaces of A and B."""
    qa, _ = np.linalg.qr(A.T)
    qb, _ = np.linalg.qr(B.T)
    return np.linalg.svd(qa.T @ qb, compute_uv=False)


def cov(X):
    Xc = np.asarray(X, np.float64) - np.asarray(X, np.float64).mean(0)
    return Xc.T @ Xc


def test_exact_low_rank_is_recovered():
    C = cov(gen.exact_rank(300, 60, 7, seed=3))
    lam, Vt = rpca.randomized_axes(C, 12, 0, 5)
    w, V = np.linalg.eigh(C)
    top = V[:, ::-1][:, :7].T
    assert np.allclose(lam[:7], w[::-1][:7], rtol=1e-10)
    assert angles_cos(Vt[:7], top).min() > 1 - 1e-12
    assert np.all(np.abs(lam[7:]) <= 1e-9 * lam[0])


def test_full_block_gives_every_eigenpair():
    C = cov(gen.gaussian(200, 40, seed=4))
    lam, Vt = rpca.randomized_axes(C, 40, 1, 9)
    w, V = np.linalg.eigh(C)
    assert np.allclose(lam, w[::-1], rtol=1e-10)
    for i in range(40):
        assert abs(abs(Vt[i] @ V[:, ::-1][:, i]) - 1) < 1e-8
    assert np.allclose(Vt @ Vt.T, np.eye(40), atol=1e-12)


def test_ritz_values_interlace():
    """Ritz values of a subspace are bounded by the true eigenvalues of the
    same rank (Cauchy interlacing): lambda_i(Q^T C Q) <= lambda_i(C)."""
    C = cov(gen.power_law(500, 80, 30, 1.0, seed=6))
    w = np.linalg.eigvalsh(C)[::-1]
    for q in (0, 1, 3):
        lam, _ = rpca.randomized_axes(C, 20, q, 2)
        assert np.all(lam <= w[:20] * (1 + 1e-12) + 1e-9)


def test_orthonormalisation_method_does_not_matter():
    """The result depends on the span only: the same steps with a symmetric
    (eigen-based) orthonormal basis in place of QR agree to rounding."""
    C = cov(gen.power_law(400, 64, 40, 0.8, seed=8))
    ell, q, seed = 24, 2, 11
    lam, Vt = rpca.randomized_axes(C, ell, q, seed)
    Om = jl_signs.jl_matrix(np.uint64(seed) ^ np.uint64(rpca.STREAM), ell, 64).T
    Q = Om
    for _ in range(q + 1):
        Y = C @ Q
        g, V = np.linalg.eigh(Y.T @ Y)
        Q = Y @ V / np.sqrt(g)
    B = Q.T @ C @ Q
    l2, W = np.linalg.eigh((B + B.T) / 2)
    o = np.argsort(-l2)
    assert np.allclose(l2[o], lam, rtol=1e-8)
    assert angles_cos((Q @ W[:, o]).T[:10], Vt[:10]).min() > 1 - 1e-8


def test_power_iterations_converge():
    C = cov(gen.power_law(600, 100, 60, 0.7, seed=12))
    w, V = np.linalg.eigh(C)
    top = V[:, ::-1][:, :10].T
    errs = []
    for q in (0, 1, 2, 4):
        _, Vt = rpca.randomized_axes(C, 20, q, 3)
        errs.append(1 - angles_cos(Vt[:10], top).min())
    assert errs[-1] < 1e-3 * errs[0]
    assert all(b <= a * 1.0001 + 1e-15 for a, b in zip(errs, errs[1:]))
