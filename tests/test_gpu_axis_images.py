"""A fit keeps the FP64 images of its maps' principal-axis rows (the leading
rows of every map of Algorithm 1 and of the PCA family) across its probes and
forms only the other rows' images per probe.  An image entry depends only on
its point and its map row, never on the product that formed it, so the fit's
certificate must equal, bit for bit, the certificate of its returned map
formed from scratch: the same exact maximum and the same pair.  The clouds
make the search grow the kept block (a probe above every earlier one), shrink
it, reach the full dimension, and recompute the axes (randomized PCA)."""
import numpy as np
import pytest
import torch

from paper_1609_05388_amd import gen

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def same_as_from_scratch(gpu_lib, Xd, f):
    c = f["cert"]
    assert c["certified"] == 1
    g = gpu_lib.certify_map(Xd, f["Pi"].contiguous())
    assert g["certified"] == 1
    assert g["max_distortion"] == c["max_distortion"]
    assert (g["i"], g["j"]) == (c["i"], c["j"])


@pytest.mark.parametrize("family", ["adagio", "pca"])
def test_fit_low_rank_matches_map_certified_from_scratch(gpu_lib, family):
    """Low-rank pixels: r well below d / 2, the probes shrink the block."""
    X = gen.low_rank_pixels(n=1500, d=96, rank=10, seed=31)
    print("axis images, low rank, family %s" % family, flush=True)
    Xd = dev(X)
    f = gpu_lib.fit(Xd, 0.1, gen.JL_SEED, family=family)
    assert 1 <= f["r"] < 96
    same_as_from_scratch(gpu_lib, Xd, f)


def test_fit_isotropic_grows_the_kept_block(gpu_lib):
    """An isotropic cloud needs r above d / 2: after the first probe (at
    d / 2) the search probes larger maps, whose axis rows extend the kept
    block."""
    X = gen.gaussian(1200, 40, seed=32)
    print("axis images, isotropic", flush=True)
    Xd = dev(X)
    f = gpu_lib.fit(Xd, 0.1, gen.JL_SEED)
    assert f["r"] > 20
    same_as_from_scratch(gpu_lib, Xd, f)


def test_fit_randomized_pca_resets_the_kept_block(gpu_lib):
    """The randomized PCA recomputes its axes when a probe needs more
    directions than its block holds; images of the old axes must not be
    reused."""
    X = gen.low_rank_pixels(n=1500, d=128, rank=40, seed=33)
    print("axis images, randomized PCA", flush=True)
    Xd = dev(X)
    f = gpu_lib.fit(Xd, 0.1, gen.JL_SEED, pca="randomized")
    same_as_from_scratch(gpu_lib, Xd, f)
