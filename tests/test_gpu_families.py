"""Map families of Table 3 (Sec. 4.4) on the GPU: the same certified search
over the PCA-only and JL-only maps, against the oracle's search over its own
family maps (same r, same certified maximum)."""
import numpy as np
import pytest
import torch

from oracle import embedding, pca as opca, search
from paper_1609_05388_amd import gen

pytestmark = pytest.mark.gpu
TOL = 1e-5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def c1():
    X = gen.low_rank_pixels()
    _, _, lam, Vt = opca.pca(X)
    return X, (lam, Vt)


@pytest.mark.parametrize("family,eps", [("pca", 0.1), ("pca", 0.2), ("jl", 0.2), ("jl", 0.4)])
def test_family_fit_parity_c1(gpu_lib, c1, family, eps):
    X, principal = c1
    want = search.fit(X, eps, gen.JL_SEED, principal=principal, family=family)
    got = gpu_lib.fit(dev(X), eps, gen.JL_SEED, family=family)
    assert got["cert"]["certified"] == 1 and got["cert"]["max_distortion"] <= eps
    near = [abs(dl - eps) for _, dl in want["probes"]]
    if min(near) > TOL:
        assert got["r"] == want["r"]
        assert abs(got["cert"]["max_distortion"] - want["cert"]["max"]) <= TOL
    if family == "pca":
        assert got["s"] == got["r"] and got["k"] == 0
    else:
        assert got["s"] == 0


def test_family_maps_are_the_oracle_maps(gpu_lib, c1):
    """The PCA-only map spans the oracle's top-r subspace; the JL-only map is
    the oracle's sign matrix (FP32 rounding of +-1/sqrt(r)); the identity at
    r = d."""
    X, (lam, Vt) = c1
    Xd = dev(X)
    g = gpu_lib.fit(Xd, 0.2, gen.JL_SEED, family="jl")
    r = g["r"]
    want = embedding.jl_map(X.shape[1], r, gen.JL_SEED).astype(np.float32)
    assert np.array_equal(g["Pi"].cpu().numpy(), want)
    p = gpu_lib.fit(Xd, 0.2, gen.JL_SEED, family="pca")
    P = p["Pi"].cpu().numpy().astype(np.float64)
    Vo = Vt[:p["r"]]
    cos = np.linalg.svd(P @ Vo.T, compute_uv=False)
    assert cos.min() > 1 - 1e-6


@pytest.mark.parametrize("r", [1, 37, 96])
def test_project_family_maps(gpu_lib, c1, r):
    """Fixed-r maps of the three families from the library's own axes: the
    Algorithm 1 map equals adagio_project_axes's bit for bit, the PCA map is
    Vt's top r rows, the JL map the oracle's sign matrix."""
    X, (lam, Vt) = c1
    _, Vg = gpu_lib.pca(dev(X))
    a = gpu_lib.project_family(Vg, r, "adagio", gen.JL_SEED)
    assert torch.equal(a, gpu_lib.project_axes(Vg, r, gen.JL_SEED))
    p = gpu_lib.project_family(Vg, r, "pca", gen.JL_SEED).cpu().numpy()
    assert np.array_equal(p, Vg[:r].cpu().numpy().astype(np.float32))
    j = gpu_lib.project_family(Vg, r, "jl", gen.JL_SEED).cpu().numpy()
    want = embedding.jl_map(X.shape[1], r, gen.JL_SEED).astype(np.float32) if r < X.shape[1] else np.eye(r, dtype=np.float32)
    assert np.array_equal(j, want)
