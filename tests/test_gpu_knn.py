"""Exact kNN queries and the majority vote (the applications of Secs. 4.6 and 4.7) on the GPU
against the oracle: indices and FP64 distances bit for bit (both sides sum the
same squares in the same order and order ties by index)."""
import numpy as np
import pytest
import torch

from oracle import knn as oknn
from paper_1609_05388_amd import gen

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check(gpu_lib, Q, D, k, exclude_self=False, rows=None):
    idx, dist, st = gpu_lib.knn(dev(Q), dev(D), k, exclude_self=exclude_self)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    sel = np.arange(len(Q)) if rows is None else rows
    wi, wd = oknn.knn(Q[sel], D, k, exclude_self=False) if not exclude_self else _excl(Q, D, k, sel)
    assert np.array_equal(idx[sel], wi), "indices differ"
    assert np.array_equal(dist[sel], wd), "distances differ"
    return st


def _excl(Q, D, k, sel):
    """exclude_self on a subset of queries: query i skips row i."""
    out_i, out_d = [], []
    for i in sel:
        d2 = oknn.sq_dists(Q[i:i + 1], D)[0]
        d2[i] = np.inf
        o = np.lexsort((np.arange(len(D)), d2))[:k]
        out_i.append(o)
        out_d.append(d2[o])
    return np.array(out_i), np.array(out_d)


@pytest.mark.parametrize("nq,nd,m,k", [
    (300, 5000, 128, 10),      # ragged database tail, SIFT width
    (257, 3001, 7, 1),         # ragged queries and width
    (130, 4000, 20, 30),       # 30-NN, embedded width
    (5, 40, 3, 32),            # database smaller than one tile and than the kept list
    (129, 700, 1, 5),          # one coordinate: many equal distances
])
def test_knn_matches_oracle(gpu_lib, nq, nd, m, k):
    rng = np.random.default_rng(nq * 7 + nd)
    D = (rng.standard_normal((nd, m)) * 3 + 1).astype(np.float32)
    Q = (rng.standard_normal((nq, m)) * 3 + 1).astype(np.float32)
    if m == 1:
        D = np.round(D)
        Q = np.round(Q)
    check(gpu_lib, Q, D, k)


def test_knn_graph_excludes_self(gpu_lib):
    X = gen.gaussian(2000, 16, seed=31)
    X = gen.with_duplicates(X, 50, seed=31)            # equal rows are ordinary neighbours
    check(gpu_lib, X, X, 30, exclude_self=True)


@pytest.mark.parametrize("nq,nd,m,k", [
    (100, 300, 9, 7),          # query block ends inside the first database tile
    (33, 33, 5, 32),           # k = nd - 1: every other row is an answer
    (200, 1000, 130, 12),      # width past one 128-column chunk, queries span blocks
])
def test_knn_exclude_self_ragged(gpu_lib, nq, nd, m, k):
    rng = np.random.default_rng(nd + m)
    D = rng.standard_normal((nd, m)).astype(np.float32)
    check(gpu_lib, D[:nq].copy(), D, k, exclude_self=True)


def test_knn_sift_integer_ties(gpu_lib):
    """Integer SIFT-shaped descriptors: FP32 estimates are exact, distances
    tie often; the answer still matches (distance, index) order exactly."""
    D, dl, Q, qi = gen.sift_shaped(buildings=12, photos=4, per_photo=120, per_query=40, proto=60, clutter=200)
    st = check(gpu_lib, Q, D, 10)
    assert st["splits"] >= 1


def test_knn_duplicate_cluster_falls_back(gpu_lib):
    """40 copies of one point: the 32 kept candidates cannot prove the
    answer, the FP64 brute force gives it (smallest indices first)."""
    rng = np.random.default_rng(4)
    D = rng.standard_normal((3000, 24)).astype(np.float32) * 10
    D[100:3000:70] = D[5]                                # 42 more copies of row 5, spread out
    Q = D[[5, 6, 7]] + np.float32(1e-3)
    st = check(gpu_lib, Q, D, 30)
    assert st["n_fallback"] >= 1


def test_knn_sift_shaped_full_size_sampled(gpu_lib):
    """The retrieval workload at its full size (402,000 x 128 database, 20,100
    queries, k = 10), in the launch configuration the benchmark times: 24
    sampled queries against the oracle, every answer sorted and in range."""
    D, dl, Q, qi = gen.sift_shaped()
    rows = np.random.default_rng(2).choice(len(Q), 24, replace=False)
    idx, dist, st = gpu_lib.knn(dev(Q), dev(D), 10)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    wi, wd = oknn.knn(Q[rows], D, 10)
    assert np.array_equal(idx[rows], wi) and np.array_equal(dist[rows], wd)
    assert idx.min() >= 0 and idx.max() < len(D)
    assert np.all(np.diff(dist, axis=1) >= 0)
    assert st["splits"] >= 1


def test_vote_matches_oracle(gpu_lib):
    rng = np.random.default_rng(8)
    nd, n_labels = 5000, 37
    d_label = rng.integers(0, n_labels, nd).astype(np.int32)
    nn = rng.integers(0, nd, (1003, 10)).astype(np.int32)
    q_group = np.arange(1003) // 100                     # last group holds 3 queries
    want, _ = oknn.vote(nn, d_label, q_group, n_labels)
    got = gpu_lib.knn_vote(dev(nn), dev(d_label), n_labels, 100).cpu().numpy()
    assert np.array_equal(got, want)
    nn[:] = nn[0, 0]                                     # every group votes for one label
    got = gpu_lib.knn_vote(dev(nn), dev(d_label), n_labels, 100).cpu().numpy()
    assert np.all(got == d_label[nn[0, 0]])


def test_retrieval_pipeline_small(gpu_lib):
    """kNN then vote on a small SIFT-shaped workload: same labels, same
    accuracy as the oracle's pipeline."""
    D, dl, Q, qi = gen.sift_shaped(buildings=20, photos=4, per_photo=60, per_query=25, proto=40, clutter=300)
    idx, _, _ = gpu_lib.knn(dev(Q), dev(D), 10)
    got = gpu_lib.knn_vote(idx, dev(dl), 20, 25).cpu().numpy()
    wi, _ = oknn.knn(Q, D, 10)
    want, _ = oknn.vote(wi, dl, qi, 20)
    assert np.array_equal(got, want)
    assert oknn.accuracy(got, np.arange(20)) == oknn.accuracy(want, np.arange(20))


def test_knn_rejects_bad_arguments(gpu_lib):
    X = dev(gen.gaussian(100, 8))
    for kw in ({"k": 0}, {"k": 33}, {"k": 100, "exclude_self": True}):
        with pytest.raises(gpu_lib.AdagioError):
            gpu_lib.knn(X, X, **kw)
    with pytest.raises(gpu_lib.AdagioError):
        gpu_lib.knn(dev(gen.gaussian(101, 8)), X, 3, exclude_self=True)
    bad = gen.gaussian(100, 8)
    bad[7, 3] = np.nan
    with pytest.raises(gpu_lib.AdagioError):
        gpu_lib.knn(X, dev(bad), 3)
    nn = torch.full((4, 2), 100, dtype=torch.int32, device="cuda")
    with pytest.raises(gpu_lib.AdagioError):
        gpu_lib.knn_vote(nn, torch.zeros(100, dtype=torch.int32, device="cuda"), 3, 2)
