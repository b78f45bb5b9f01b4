"""The no-allocation certificate (adagio_max_distortion_noalloc) against the
allocating one (adagio_max_distortion) on the same inputs, through the C ABI:
two calls in a row, the second on a smaller cloud, so that the second reuses
the fixed scratch array the first left behind.  Both run the same kernels in
the same order, so every field of the certificate is identical; the maximum
also meets the FP64 oracle's eq. (3) within 1e-5 (argmax equal where the
oracle's runner-up gap exceeds that)."""
import numpy as np
import pytest
import torch

from oracle import certificate
from paper_1609_05388_amd import gen

pytestmark = pytest.mark.gpu

TOL = 1e-5
FIELDS = ("max_distortion", "i", "j", "side", "certified", "runner_up", "i2", "j2", "bound_rest", "n_rescored",
          "n_pairs", "n_flagged_tiles")


def _case(seed, n, d, rank, r):
    X = gen.low_rank_pixels(n=n, d=d, rank=rank, seed=seed)
    rng = np.random.default_rng(seed + 1)
    Pi = (rng.standard_normal((r, d)) / np.sqrt(r)).astype(np.float32)
    Y = (X.astype(np.float64) @ Pi.T.astype(np.float64)).astype(np.float32)
    return X, Y


@pytest.mark.parametrize("calls", [[(31, 3000, 200, 12, 48), (32, 777, 90, 9, 21)]])
def test_noalloc_certificate_matches_allocating_one(gpu_lib, calls):
    for seed, n, d, rank, r in calls:
        print("no-alloc certificate: n=%d d=%d r=%d seed=%d" % (n, d, r, seed), flush=True)
        X, Y = _case(seed, n, d, rank, r)
        Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
        got = gpu_lib.max_distortion_noalloc(Xd, Yd)
        ref = gpu_lib.max_distortion(Xd, Yd)
        for f in FIELDS:
            assert got[f] == ref[f], (f, got, ref)
        assert got["certified"] == 1
        want = certificate.certify(X, Y)
        assert abs(got["max_distortion"] - want["max"]) <= TOL, (got, want)
        if want["max"] - want["runner_up"] > TOL:
            assert (got["i"], got["j"]) == (want["i"], want["j"])


def test_noalloc_refuses_clouds_beyond_its_scratch(gpu_lib):
    X = torch.zeros((20000, 784), dtype=torch.float32, device="cuda")
    Y = torch.zeros((20000, 256), dtype=torch.float32, device="cuda")
    with pytest.raises(gpu_lib.AdagioError) as e:
        gpu_lib.max_distortion_noalloc(X, Y)
    assert e.value.code == -5
