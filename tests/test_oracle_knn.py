"""Pins of the oracle's exact kNN and majority vote (the applications of Secs. 4.6 and 4.7)
against what the definitions fix: exact rational brute force on tiny integer
inputs (ties included), scikit-learn's brute-force search, exact invariances,
self-matches, and hand-worked votes."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import knn
from paper_1609_05388_amd import gen


def brute(Q, D, k, exclude_self=False):
    """Exact rational distances, Python's sort on (distance, index)."""
    out = []
    for i, q in enumerate(Q):
        cand = []
        for j, x in enumerate(D):
            if exclude_self and i == j:
                continue
            cand.append((sum((Fraction(float(a)) - Fraction(float(b))) ** 2 for a, b in zip(q, x)), j))
        cand.sort()
        out.append(cand[:k])
    return out


@pytest.mark.parametrize("exclude_self", [False, True])
def test_tiny_integer_brute_force_with_ties(exclude_self):
    rng = np.random.default_rng(5)
    D = rng.integers(-3, 4, (40, 3)).astype(np.float32)      # many equal distances
    Q = D[:12] if exclude_self else rng.integers(-3, 4, (12, 3)).astype(np.float32)
    idx, dist = knn.knn(Q, D, 7, exclude_self=exclude_self, block=5)   # block < nq: offsets matter
    want = brute(Q, D, 7, exclude_self)
    for i in range(len(Q)):
        assert [j for _, j in want[i]] == list(idx[i])
        assert [float(d) for d, _ in want[i]] == list(dist[i])


def test_matches_scikit_learn_brute_force():
    from sklearn.neighbors import NearestNeighbors
    rng = np.random.default_rng(6)
    D = rng.standard_normal((500, 17)).astype(np.float32)
    Q = rng.standard_normal((60, 17)).astype(np.float32)
    idx, dist = knn.knn(Q, D, 10)
    nn = NearestNeighbors(n_neighbors=10, algorithm="brute").fit(D.astype(np.float64))
    d_sk, i_sk = nn.kneighbors(Q.astype(np.float64))
    assert np.array_equal(idx, i_sk)
    assert np.allclose(dist, d_sk ** 2, rtol=1e-12)


def test_exact_invariances_on_integer_data():
    """Permuting coordinates and translating by an integer vector leave every
    distance (exact on small integers) and so every answer unchanged."""
    rng = np.random.default_rng(7)
    D = rng.integers(0, 50, (300, 9)).astype(np.float32)
    Q = rng.integers(0, 50, (40, 9)).astype(np.float32)
    perm = rng.permutation(9)
    t = rng.integers(-100, 100, 9).astype(np.float32)
    i1, d1 = knn.knn(Q, D, 12)
    i2, d2 = knn.knn(Q[:, perm] + t[perm], D[:, perm] + t[perm], 12)
    assert np.array_equal(i1, i2) and np.array_equal(d1, d2)


def test_self_match_and_exclusion():
    X = gen.gaussian(200, 8, seed=3)
    idx, dist = knn.knn(X, X, 3)
    assert np.array_equal(idx[:, 0], np.arange(200)) and np.all(dist[:, 0] == 0)
    idx2, dist2 = knn.knn(X, X, 2, exclude_self=True, block=64)
    assert np.array_equal(idx2, idx[:, 1:3]) and np.array_equal(dist2, dist[:, 1:3])


def test_duplicates_are_ordered_by_index():
    X = gen.gaussian(50, 4, seed=8)
    D = np.concatenate([X, X[::-1], X])            # every point three times
    idx, dist = knn.knn(X, D, 3)
    for i in range(50):
        assert list(idx[i]) == [i, 99 - i, 100 + i]
        assert np.all(dist[i] == 0)


def test_k_equal_database_size_sorts_everything():
    rng = np.random.default_rng(9)
    D = rng.standard_normal((31, 5)).astype(np.float32)
    q = rng.standard_normal((1, 5)).astype(np.float32)
    idx, dist = knn.knn(q, D, 31)
    assert sorted(idx[0]) == list(range(31)) and np.all(np.diff(dist[0]) >= 0)
    with pytest.raises(ValueError):
        knn.knn(q, D, 32)
    with pytest.raises(ValueError):
        knn.knn(D, D, 31, exclude_self=True)


def test_vote_hand_worked():
    d_label = np.array([0, 0, 1, 1, 2, 2, 3])
    # group 0: labels 1,1,2 | 0 -> 1 wins; group 1: labels 2,3 | 3,2 -> tie 2/3 -> 2
    nn = np.array([[2, 3], [4, 0], [4, 6], [6, 5]])
    pred, votes = knn.vote(nn, d_label, np.array([0, 0, 1, 1]), 4)
    assert list(pred) == [1, 2]
    assert votes.tolist() == [[1, 2, 1, 0], [0, 0, 2, 2]]
    assert knn.accuracy(pred, [1, 3]) == 0.5


def test_sift_shaped_layout():
    D, dl, Q, qi = gen.sift_shaped(buildings=5, photos=2, per_photo=30, per_query=7, proto=20, clutter=40)
    assert D.shape == (300, 128) and Q.shape == (35, 128)
    assert np.all(D == np.round(D)) and D.min() >= 0 and np.all(np.abs(np.linalg.norm(D, axis=1) - 512) < 6)
    assert list(np.bincount(dl)) == [60] * 5 and list(np.bincount(qi)) == [7] * 5
