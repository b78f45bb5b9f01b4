"""Compact D^2 cache of the precision-form fits (BF16 split and FP8 screens):
per tile the pairs' D2lo rounded down to FP16 at a power-of-two scale.  The
cache only loosens the screens' bounds (by 2^-10 relative), so a fit that
uses it must take exactly the plain FP32 fit's decisions and return the same
certificate, and the FP8-screened fit's certificate must be the oracle's for
its map.  The clouds push the cache where it can break: row norms over six
decades (many pairs' D^2 far below the scale), identical points (D2lo <= 0),
and the whole cloud scaled by powers of two far from 1 (the scale's clamp and
the exactness of the division by it)."""
import numpy as np
import pytest
import torch

from oracle import certificate, embedding
from paper_1609_05388_amd import gen

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def wide_norms(n=1500, d=64, seed=21):
    """Low-rank points whose rows are rescaled by 10^U[-3, 3], with 20
    duplicated rows."""
    rng = np.random.default_rng(seed)
    X = gen.low_rank_pixels(n=n, d=d, rank=12, seed=seed).astype(np.float64)
    X *= 10.0 ** rng.uniform(-3.0, 3.0, (n, 1))
    return gen.with_duplicates(X.astype(np.float32), 20, seed=seed)


def same_fit(a, b):
    assert a["r"] == b["r"]
    assert torch.equal(a["Pi"], b["Pi"])
    for key in ("max_distortion", "i", "j", "side", "certified"):
        assert a["cert"][key] == b["cert"][key], key


@pytest.mark.parametrize("power", [0, -40, 40])
def test_bf16x3_fit_with_cache_equals_plain(gpu_lib, power):
    X = wide_norms() * np.float32(2.0 ** power)
    print("bf16x3 fit, wide norms x 2^%d" % power, flush=True)
    Xd = dev(X)
    a = gpu_lib.fit(Xd, 0.1, gen.JL_SEED)
    b = gpu_lib.fit(Xd, 0.1, gen.JL_SEED, screen="bf16x3")
    same_fit(a, b)


@pytest.mark.parametrize("power", [0, -40, 40])
def test_fp8_fit_with_cache_certified_by_oracle(gpu_lib, power):
    X = wide_norms(seed=22) * np.float32(2.0 ** power)
    print("fp8 fit, wide norms x 2^%d" % power, flush=True)
    f = gpu_lib.fit(dev(X), 0.1, gen.JL_SEED, screen="fp8")
    c = f["cert"]
    assert c["certified"] == 1 and c["max_distortion"] <= 0.1
    Pi = f["Pi"][: f["r"]].cpu().numpy().astype(np.float64)
    want = certificate.certify(X, embedding.embed(X, Pi))
    assert abs(c["max_distortion"] - want["max"]) <= 1e-12
    if want["max"] - want["runner_up"] > 1e-12:
        assert (c["i"], c["j"]) == (want["i"], want["j"])


def test_bf16x3_fit_all_points_identical_but_two(gpu_lib):
    """A cloud of one repeated point and two others: almost every pair has
    D^2 = 0, so D2lo <= 0 and the cache's lower bound is not positive."""
    X = np.zeros((400, 16), dtype=np.float32)
    X[:] = np.linspace(-1.0, 1.0, 16, dtype=np.float32)
    X[5, 3] += 0.5
    X[300, 7] -= 0.25
    Xd = dev(X)
    a = gpu_lib.fit(Xd, 0.1, gen.JL_SEED)
    b = gpu_lib.fit(Xd, 0.1, gen.JL_SEED, screen="bf16x3")
    same_fit(a, b)


@pytest.mark.parametrize("n", [1100, 1300])
def test_precision_fits_odd_tile_count(gpu_lib, n):
    """An odd number of 128-row tiles (9 and 11): the cache fill works on
    quads of 2 x 2 tiles, so its last quad row and column hold one tile and
    read rows past the cloud (from its last row), which must not reach any
    stored block."""
    X = wide_norms(n=n, seed=n)
    print("precision fits, n = %d" % n, flush=True)
    Xd = dev(X)
    a = gpu_lib.fit(Xd, 0.1, gen.JL_SEED)
    b = gpu_lib.fit(Xd, 0.1, gen.JL_SEED, screen="bf16x3")
    same_fit(a, b)
    f = gpu_lib.fit(Xd, 0.1, gen.JL_SEED, screen="fp8")
    assert f["cert"]["certified"] == 1
    assert f["r"] == a["r"] and torch.equal(f["Pi"], a["Pi"])


@pytest.mark.parametrize("n", [1100, 1300, 1500])
def test_fp8_fit_long_image_rows(gpu_lib, n):
    """Maps with at least eight 64-column image chunks (r > 448) screen on
    256 x 256 quads of tiles; odd tile counts (9, 11 tiles) leave quads
    with rows past the cloud.  The FP8-screened fit's certificate must be the
    oracle's for its map."""
    rng = np.random.default_rng(n)
    X = gen.low_rank_pixels(n=n, d=1100, rank=300, seed=n).astype(np.float64)
    X *= 10.0 ** rng.uniform(-1.0, 1.0, (n, 1))
    X = X.astype(np.float32)
    print("fp8 fit, %d x 1100, long image rows" % n, flush=True)
    Xd = dev(X)
    f = gpu_lib.fit(Xd, 0.1, gen.JL_SEED, screen="fp8")
    assert max(f["stats"]["probe_cols"]) > 448
    c = f["cert"]
    assert c["certified"] == 1 and c["max_distortion"] <= 0.1
    Pi = f["Pi"][: f["r"]].cpu().numpy().astype(np.float64)
    want = certificate.certify(X, embedding.embed(X, Pi))
    assert abs(c["max_distortion"] - want["max"]) <= 1e-12
    if want["max"] - want["runner_up"] > 1e-12:
        assert (c["i"], c["j"]) == (want["i"], want["j"])
