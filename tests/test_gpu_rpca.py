"""Randomized PCA (Sec. 4.5's variant) on the GPU against the oracle's, and
fits that take their principal directions from it."""
import numpy as np
import pytest
import torch

from oracle import certificate, embedding, rpca
from paper_1609_05388_amd import gen

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def row_space_cos(A, B):
    qa, _ = np.linalg.qr(np.asarray(A, np.float64).T)
    qb, _ = np.linalg.qr(np.asarray(B, np.float64).T)
    return np.linalg.svd(qa.T @ qb, compute_uv=False)


@pytest.mark.parametrize("ell,q", [(60, 2), (120, 0), (120, 3)])
def test_randomized_axes_match_oracle(gpu_lib, ell, q):
    X = gen.low_rank_pixels()
    lam, Vt = gpu_lib.pca_randomized(dev(X), ell, q, gen.JL_SEED)
    lo, Vo = rpca.randomized_pca(X, ell, q, gen.JL_SEED)
    lam, Vt = lam.cpu().numpy(), Vt.cpu().numpy()
    k = ell // 2
    assert np.allclose(lam[:k], lo[:k], rtol=1e-9)
    assert row_space_cos(Vt[:k], Vo[:k]).min() > 1 - 1e-9
    assert np.allclose(Vt @ Vt.T, np.eye(ell), atol=1e-10)


def test_full_block_is_the_exact_eigenbasis(gpu_lib):
    X = gen.gaussian(700, 96, seed=21)
    lam, Vt = gpu_lib.pca_randomized(dev(X), 96, 1, 5)
    w = np.linalg.eigvalsh(np.cov(X.astype(np.float64).T) * (len(X) - 1))[::-1]
    assert np.allclose(lam.cpu().numpy(), w, rtol=1e-9)


@pytest.mark.parametrize("search", ["bisect", "learned"])
def test_fit_with_randomized_pca_is_certified(gpu_lib, search):
    """The certificate is exact for the map the fit returns, whatever its
    principal directions: the oracle re-certifies that map."""
    X = gen.low_rank_pixels()
    kw = {}
    if search == "learned":
        from paper_1609_05388_amd import learned
        import os
        if not os.path.exists(learned.PREDICTOR):
            pytest.skip("no trained predictor committed")
        kw = {"search": "learned", "predictor": learned.load_predictor()}
    f = gpu_lib.fit(dev(X), 0.1, gen.JL_SEED, pca="randomized", pca_iters=2, **kw)
    c = f["cert"]
    assert c["certified"] == 1 and c["max_distortion"] <= 0.1
    Pi = f["Pi"].cpu().numpy().astype(np.float64)
    want = certificate.certify(X, embedding.embed(X, Pi))
    assert abs(want["max"] - c["max_distortion"]) <= 1e-5
    # against the same search with exact PCA (the learned search returns the
    # prediction when it certifies, so there both give the predicted r)
    exact = gpu_lib.fit(dev(X), 0.1, gen.JL_SEED, **kw)
    assert abs(f["r"] - exact["r"]) <= max(4, exact["r"] // 10)
