"""Precision form: the BF16 split-precision screen (x = hi + lo, three BF16
MFMA products, FP32 accumulation) with rigorous bounds and exact FP64
rescoring.  Its certificate equals the oracle's to FP64 rounding, and a fit
with it takes exactly the decisions of the plain FP32 fit."""
import numpy as np
import pytest
import torch

from oracle import certificate, embedding, pca as opca
from paper_1609_05388_amd import gen

pytestmark = pytest.mark.gpu
TOL_PRECISION = 1e-4   # the precision form's stated tolerance on the max distortion
TOL = 1e-5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check(got, want, tol):
    assert got["certified"] == 1
    err = abs(got["max_distortion"] - want["max"])
    assert err <= tol, (got, want)
    if want["max"] - want["runner_up"] > tol:
        assert (got["i"], got["j"]) == (want["i"], want["j"])
    return err


def test_bf16x3_certificate_parity_c1(gpu_lib):
    X = gen.low_rank_pixels()
    _, _, _, Vt = opca.pca(X)
    for r in (93, 213, 391):
        Pi32 = embedding.adagio_map(Vt, r, gen.JL_SEED).astype(np.float32)
        want = certificate.certify(X, embedding.embed(X, Pi32.astype(np.float64)))
        got = gpu_lib.certify_map(dev(X), dev(Pi32), screen="bf16x3")
        err = check(got, want, TOL_PRECISION)
        assert err <= 1e-12   # exact rescoring: FP64 rounding only
        Y = embedding.embed(X, Pi32.astype(np.float64)).astype(np.float32)
        g2 = gpu_lib.max_distortion(dev(X), dev(Y), screen="bf16x3")
        check(g2, certificate.certify(X, Y), TOL)


@pytest.mark.parametrize("n,d,r", [(2, 1, 1), (65, 7, 3), (129, 64, 20), (300, 100, 99), (700, 33, 5)])
def test_bf16x3_ragged(gpu_lib, n, d, r):
    X = gen.gaussian(n, d, seed=n + 7 * d)
    Pi = gen.gaussian(r, d, seed=r + 3) / np.float32(np.sqrt(d))
    want = certificate.certify(X, embedding.embed(X, Pi.astype(np.float64)))
    got = gpu_lib.certify_map(dev(X), dev(Pi), screen="bf16x3")
    check(got, want, TOL)


def test_bf16x3_offset_and_duplicates(gpu_lib):
    X = gen.with_duplicates(gen.gaussian(500, 40, seed=3, scale=0.02, offset=30.0), 30)
    Pi = gen.gaussian(12, 40, seed=4)
    Y = embedding.embed(X, Pi.astype(np.float64)).astype(np.float32)
    got = gpu_lib.max_distortion(dev(X), dev(Y), screen="bf16x3")
    check(got, certificate.certify(X, Y), TOL)


@pytest.mark.parametrize("eps", [0.05, 0.1, 0.2])
def test_bf16x3_fit_equals_plain_c1(gpu_lib, eps):
    X = dev(gen.low_rank_pixels())
    a = gpu_lib.fit(X, eps, gen.JL_SEED)
    b = gpu_lib.fit(X, eps, gen.JL_SEED, screen="bf16x3")
    assert a["r"] == b["r"]
    assert torch.equal(a["Pi"], b["Pi"])
    for key in ("max_distortion", "i", "j", "side", "certified"):
        assert a["cert"][key] == b["cert"][key]


def test_bf16x3_fit_equals_plain_mnist_shaped(gpu_lib):
    X = dev(gen.mnist_shaped())
    a = gpu_lib.fit(X, 0.1, gen.JL_SEED)
    b = gpu_lib.fit(X, 0.1, gen.JL_SEED, screen="bf16x3")
    assert a["r"] == b["r"]
    assert torch.equal(a["Pi"], b["Pi"])
    assert a["cert"]["max_distortion"] == b["cert"]["max_distortion"]
    assert (a["cert"]["i"], a["cert"]["j"]) == (b["cert"]["i"], b["cert"]["j"])
