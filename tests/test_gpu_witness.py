"""Refutation by witness pairs in the fit's search: eq. (3) is a maximum over
pairs, so one pair whose exact eq. (2) value exceeds eps fails a probe's map
without its all-pairs screen.  The fit keeps a pool of the worst record pairs
of its earlier certificates (kind 3) and stops a screen at a pair that its
bounds prove above eps (kind 4); the result must be the one of the search
that certifies every probe in full, probe for probe."""
import numpy as np
import pytest
import torch

from oracle import certificate as ocert
from oracle import embedding as oemb
from oracle import search
from paper_1609_05388_amd import gen

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = [
    ("c1", 0.1, "f32"),
    ("c1", 0.05, "f32"),
    ("c1", 0.2, "bf16x3"),
    ("mnist", 0.1, "f32"),
    ("mnist", 0.1, "fp8"),
]


def cloud(name):
    if name == "c1":
        return gen.low_rank_pixels()
    return gen.mnist_shaped(n=3000)


@pytest.mark.parametrize("name,eps,screen,family", [c + ("adagio",) for c in CASES] + [
    ("mnist", 0.1, "f32", "pca"),      # Table 3's PCA-only maps
    ("c1", 0.2, "f32", "jl"),          # JL-only maps: no PCA, the cache fill starts at once
])
def test_witness_search_same_result(gpu_lib, name, eps, screen, family):
    X = cloud(name)
    a = gpu_lib.fit(dev(X), eps, gen.JL_SEED, screen=screen, family=family)
    b = gpu_lib.fit(dev(X), eps, gen.JL_SEED, screen=screen, family=family, witness=False)
    assert a["r"] == b["r"]
    assert torch.equal(a["Pi"], b["Pi"])
    assert a["cert"] == b["cert"]
    sa, sb = a["stats"], b["stats"]
    assert sb["n_refuted"] == 0 and 3 not in sb["probe_gram"] and 4 not in sb["probe_gram"]
    # the point-Gram cache is filled beside the PCA and every screen of the
    # search's own precision loads it
    for st in (sa, sb):
        assert st["t_gram_ms"] > 0
        assert 0 not in st["probe_gram"] and 1 not in st["probe_gram"] or screen == "fp8"
    # the same probes in the same order; each refuted one replaces a certificate
    assert sa["probe_r"] == sb["probe_r"]
    assert sa["n_certificates"] + sa["n_refuted"] == sb["n_certificates"]
    assert sa["probe_gram"].count(3) + sa["probe_gram"].count(4) == sa["n_refuted"]
    for k, g in enumerate(sa["probe_gram"]):
        full = sb["probe_delta"][k]
        if g in (3, 4):
            # an attained value above eps, at most the probe's exact maximum
            assert eps < sa["probe_delta"][k] <= full + 1e-9
            assert full > eps
        else:
            assert sa["probe_delta"][k] == full


def test_witness_values_against_oracle(gpu_lib):
    """Failing probes get refuted on this cloud; each witness value is an
    exact distortion of a pair under that probe's map (the library's own map
    at r, rebuilt from its principal axes), so it lies above eps and at most
    at the oracle's maximum for that map."""
    X = gen.mnist_shaped(n=3000)
    eps = 0.1
    a = gpu_lib.fit(dev(X), eps, gen.JL_SEED)
    st = a["stats"]
    assert st["n_refuted"] >= 2
    _, Vt = gpu_lib.pca(dev(X))
    for r, dl, g in zip(st["probe_r"], st["probe_delta"], st["probe_gram"]):
        if g not in (3, 4):
            continue
        Pi = gpu_lib.project_axes(Vt, r, gen.JL_SEED).cpu().numpy()
        want = ocert.certify(X, oemb.embed(X, Pi))
        assert eps < dl <= want["max"] + 1e-9, r


@pytest.mark.parametrize("n,d", [(2, 1), (2, 5), (3, 2), (7, 4), (130, 3)])
@pytest.mark.parametrize("screen", ["f32", "bf16x3", "fp8"])
def test_witness_search_tiny_clouds(gpu_lib, n, d, screen):
    """Clouds of one tile (or a single pair): a pool of at most a few pairs,
    early stops on tiny screens, the cache filled with one or two tiles.  The
    search visits the oracle's probes and ends at its r and maximum."""
    rng = np.random.default_rng(100 * n + d)
    X = (rng.standard_normal((n, d)) * np.linspace(1.0, 0.2, d)).astype(np.float32)
    got = gpu_lib.fit(dev(X), 0.1, gen.JL_SEED, screen=screen)
    ref = gpu_lib.fit(dev(X), 0.1, gen.JL_SEED, screen=screen, witness=False)
    assert got["r"] == ref["r"] and torch.equal(got["Pi"], ref["Pi"]) and got["cert"] == ref["cert"]
    want = search.fit(X, 0.1, gen.JL_SEED)
    near = [abs(v - 0.1) for _, v in want["probes"]]
    if not near or min(near) > 1e-5:
        assert got["r"] == want["r"]
        assert abs(got["cert"]["max_distortion"] - want["cert"]["max"]) <= 1e-5
        # the same probes (an FP8 fit then certifies its result once more)
        wr = [r for r, _ in want["probes"]]
        assert got["stats"]["probe_r"][:len(wr)] == wr
