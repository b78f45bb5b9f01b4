"""Pins of the FP64 oracle against facts the paper and mathematics fix.

Each test checks the oracle against something other than itself: published
known answers, closed forms, invariants stated or used in the paper,
brute force on tiny inputs, and library routines.  ``test_oracle_mutations``
shows that plausible mistakes planted in the oracle fail these pins.
"""
import itertools
import os

import numpy as np
import pytest
from scipy.spatial.distance import pdist

from oracle import certificate, embedding, jl_signs, pca, search
from paper_1609_05388_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- JL signs
def test_splitmix64_known_answers():
    """Published SplitMix64 reference outputs for seed 0."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    t = np.array([int(a) for a, _ in rows], dtype=np.uint64)
    want = [int(b, 16) for _, b in rows]
    got = [int(v) for v in jl_signs.splitmix64_output(0, t)]
    assert got == want


def test_sign_matrix_counter_layout():
    """b[a, l] is bit 63 of output number (a * 2^32 + l + 1); rows nest in k."""
    seed = 77
    B = jl_signs.sign_matrix(seed, 3, 5)
    for a in range(3):
        for l in range(5):
            z = int(jl_signs.splitmix64_output(seed, np.uint64((a << 32) + l + 1)))
            assert B[a, l] == (1.0 if z >> 63 == 0 else -1.0)
    assert np.array_equal(jl_signs.sign_matrix(seed, 2, 5), B[:2])


def test_sign_balance_binomial_band():
    """Lemma 1: entries are uniform +-1; the count of +1 over N draws stays
    within 5 sigma of N/2, and rows are uncorrelated."""
    B = jl_signs.sign_matrix(5388, 400, 784)
    N = B.size
    plus = (B > 0).sum()
    assert abs(plus - N / 2) < 5 * np.sqrt(N / 4)
    G = (B @ B.T) / 784.0
    off = G[~np.eye(400, dtype=bool)]
    assert np.abs(off).max() < 6 / np.sqrt(784)
    assert np.allclose(np.diag(G), 1.0)


def test_jl_moments_rademacher():
    """For S with iid +-1/sqrt(k) entries: E||Sv||^2 = ||v||^2 and
    Var||Sv||^2 = (2/k)(||v||^4 - sum v_l^4).  Checked over 400 seeds."""
    rng = np.random.default_rng(3)
    d, k = 64, 16
    v = rng.standard_normal(d)
    vals = np.array([np.sum((jl_signs.jl_matrix(seed, k, d) @ v) ** 2) for seed in range(400)])
    nv2 = v @ v
    var = 2.0 / k * (nv2 ** 2 - np.sum(v ** 4))
    assert abs(vals.mean() - nv2) < 5 * np.sqrt(var / len(vals))
    assert 0.7 * var < vals.var() < 1.4 * var


# ------------------------------------------------------------ covariance
def test_covariance_equals_pairwise_secant_sum():
    """sum_i (x_i - mu)(x_i - mu)^T = (1/2n) sum_{i,j} (x_i - x_j)(x_i - x_j)^T,
    by brute force over all ordered pairs."""
    X = gen.gaussian(37, 9, seed=11, offset=3.0).astype(np.float64)
    mu, C, _, _ = pca.pca(X)
    n = X.shape[0]
    B = np.zeros((9, 9))
    for i in range(n):
        for j in range(n):
            v = X[i] - X[j]
            B += np.outer(v, v)
    assert np.allclose(C, B / (2 * n), rtol=1e-12, atol=1e-10)
    assert np.allclose(mu, [X[:, l].sum() / n for l in range(9)])


def test_covariance_translation_invariant_psd():
    X = gen.gaussian(50, 12, seed=5).astype(np.float64)
    _, C1, lam, _ = pca.pca(X)
    _, C2, _, _ = pca.pca(X + 100.0 * np.arange(12))
    assert np.allclose(C1, C2, atol=1e-8)
    assert np.allclose(C1, C1.T)
    assert lam.min() > -1e-10 * lam.max()


# ---------------------------------------------------------- eigensolve
def _jacobi_eig(A, sweeps=30):
    """Independent cyclic Jacobi (textbook, Golub & Van Loan 8.5) for pins."""
    A = A.copy()
    n = A.shape[0]
    V = np.eye(n)
    for _ in range(sweeps):
        off = np.sqrt(np.sum(A ** 2) - np.sum(np.diag(A) ** 2))
        if off < 1e-15 * np.linalg.norm(A):
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                if A[p, q] == 0.0:
                    continue
                tau = (A[q, q] - A[p, p]) / (2 * A[p, q])
                t = np.sign(tau) / (abs(tau) + np.sqrt(1 + tau * tau)) if tau != 0 else 1.0
                c = 1 / np.sqrt(1 + t * t)
                s = t * c
                J = np.eye(n)
                J[p, p] = J[q, q] = c
                J[p, q] = s
                J[q, p] = -s
                A = J.T @ A @ J
                V = V @ J
    return np.diag(A), V


def test_principal_axes_residual_and_order():
    X = gen.low_rank_pixels(n=300, d=48, rank=6, seed=2)
    _, C, lam, Vt = pca.pca(X)
    V = Vt.T
    assert np.linalg.norm(C @ V - V * lam) <= 1e-12 * np.linalg.norm(C)
    assert np.linalg.norm(Vt @ V - np.eye(48)) <= 1e-13 * 48
    assert np.all(np.diff(lam) <= 0)


def test_principal_axes_match_independent_jacobi():
    """Top-s projector agrees with a textbook Jacobi eigensolver where the
    eigengap at s is not tiny."""
    X = gen.low_rank_pixels(n=200, d=16, rank=5, seed=4).astype(np.float64)
    _, C, lam, Vt = pca.pca(X)
    w, V = _jacobi_eig(C)
    order = np.argsort(-w)
    w, V = w[order], V[:, order]
    assert np.allclose(w, lam, rtol=1e-10, atol=1e-10 * lam[0])
    for s in range(1, 16):
        if lam[s - 1] - lam[s] > 1e-6 * lam[0]:
            Pa = Vt[:s].T @ Vt[:s]
            Pb = V[:, :s] @ V[:, :s].T
            assert np.linalg.norm(Pa - Pb, 2) < 1e-9


def test_pca_minimises_eq4():
    """Eq. (4): on centred data the top-s principal projector minimises
    sum_{x,y} (||x-y||^2 - ||Pi x - Pi y||^2) over rank-s orthogonal projections."""
    X = gen.low_rank_pixels(n=60, d=20, rank=4, seed=9).astype(np.float64)
    _, _, _, Vt = pca.pca(X)
    diffs = (X[:, None, :] - X[None, :, :]).reshape(-1, 20)

    def loss(P):
        return np.sum(diffs ** 2) - np.sum((diffs @ P.T) ** 2)

    s = 5
    best = loss(Vt[:s])
    rng = np.random.default_rng(0)
    for _ in range(50):
        Q = np.linalg.qr(rng.standard_normal((20, s)))[0].T
        assert loss(Q) >= best - 1e-9
    assert loss(Vt[-s:]) > best
    assert loss(Vt[1:s + 1]) >= best - 1e-9


# ------------------------------------------------------------------- map
def test_split_rule():
    """Sec. 4.1: floor(r/2) principal components, ceil(r/2) JL rows; r = d is
    the no-reduction case."""
    assert embedding.split(1, 10) == (0, 1)
    assert embedding.split(2, 10) == (1, 1)
    assert embedding.split(3, 10) == (1, 2)
    assert embedding.split(9, 10) == (4, 5)
    assert embedding.split(10, 10) == (10, 0)
    with pytest.raises(ValueError):
        embedding.split(0, 10)


def test_map_structure():
    """P P^T = I (Algorithm 1's orthonormal P); the JL part annihilates the
    principal subspace (S Q P^T = 0) and equals S on its complement."""
    X = gen.low_rank_pixels(n=120, d=40, rank=8, seed=6)
    _, _, _, Vt = pca.pca(X)
    r = 15
    Pi = embedding.adagio_map(Vt, r, 21)
    s, k = embedding.split(r, 40)
    P, SQ = Pi[:s], Pi[s:]
    assert np.allclose(P @ P.T, np.eye(s), atol=1e-13)
    assert np.abs(SQ @ P.T).max() < 1e-13
    S = jl_signs.jl_matrix(21, k, 40)
    tail = Vt[s:]
    w = tail.T @ np.random.default_rng(1).standard_normal(40 - s)
    assert np.allclose(SQ @ w, S @ w, atol=1e-12)
    assert np.allclose(np.abs(S), 1 / np.sqrt(k))


def test_pythagoras_in_theorem2():
    """Proof of Thm. 2: ||v||^2 = ||Pv||^2 + ||Qv||^2 and
    ||Pi v||^2 = ||Pv||^2 + ||S Q v||^2 where S Q v is S applied to the
    residual v - P^T P v."""
    X = gen.low_rank_pixels(n=80, d=30, rank=5, seed=8).astype(np.float64)
    _, _, _, Vt = pca.pca(X)
    Pi = embedding.adagio_map(Vt, 11, 3)
    s, k = embedding.split(11, 30)
    P = Vt[:s]
    S = jl_signs.jl_matrix(3, k, 30)
    for (i, j) in [(0, 1), (5, 17), (40, 79)]:
        v = X[i] - X[j]
        resid = v - P.T @ (P @ v)
        assert np.isclose(v @ v, np.sum((P @ v) ** 2) + resid @ resid, rtol=1e-12)
        assert np.isclose(np.sum((Pi @ v) ** 2), np.sum((P @ v) ** 2) + np.sum((S @ resid) ** 2), rtol=1e-12)


def test_full_dimension_is_isometry():
    """r = d: no reduction, zero distortion."""
    X = gen.gaussian(90, 24, seed=12)
    _, _, _, Vt = pca.pca(X)
    c = search.distortion_of_map(X, embedding.adagio_map(Vt, 24, 1))
    assert c["max"] <= 1e-12


def test_exact_rank_data_has_zero_distortion():
    """Points on a q-dim affine subspace: with s >= q principal rows every
    secant lies in span(P), the JL rows see Q v = 0, and Pi is an isometry on
    the cloud."""
    q = 6
    X = gen.exact_rank(70, 32, q, seed=13).astype(np.float64)
    _, _, _, Vt = pca.pca(X)
    for r in (2 * q, 2 * q + 1, 20):
        c = search.distortion_of_map(X, embedding.adagio_map(Vt, r, 99))
        assert c["max"] < 1e-9, r


def test_pca_only_distortion_bound():
    """Sec. 3, "PCA and distance distortion": with P the top-s principal
    projector, 0 <= 1 - ||P(x-y)|| / ||x-y|| <= min(2 sigma_{s+1} / ||x-y||, 1)
    where sigma are the singular values of the centred data."""
    X = gen.low_rank_pixels(n=150, d=40, rank=5, noise=0.1, seed=14).astype(np.float64)
    _, _, lam, Vt = pca.pca(X)
    for s in (1, 3, 5, 10):
        P = Vt[:s]
        sig = np.sqrt(max(lam[s], 0.0))
        for i in range(0, 150, 7):
            for j in range(i + 1, 150, 5):
                v = X[i] - X[j]
                nv = np.linalg.norm(v)
                if nv == 0:
                    continue
                dist = 1 - np.linalg.norm(P @ v) / nv
                assert -1e-12 <= dist <= min(2 * sig / nv, 1.0) + 1e-12


# ----------------------------------------------------------- certificate
def _pdist_certificate(X, Y):
    D = pdist(np.asarray(X, np.float64))
    E = pdist(np.asarray(Y, np.float64))
    ok = D > 0
    dist = np.abs(E[ok] / D[ok] - 1)
    return dist.max(), dist


def test_certificate_matches_scipy_pdist():
    X = gen.gaussian(45, 10, seed=15)
    Y = X.astype(np.float64) @ np.random.default_rng(2).standard_normal((10, 4))
    c = certificate.certify(X, Y)
    best, dist = _pdist_certificate(X, Y)
    assert abs(c["max"] - best) < 1e-14
    assert abs(c["runner_up"] - np.sort(dist)[-2]) < 1e-14
    assert c["n_pairs"] == 45 * 44 // 2


def test_certificate_brute_force_and_argmax():
    X = gen.gaussian(12, 5, seed=16).astype(np.float64)
    Y = X @ np.random.default_rng(5).standard_normal((5, 3))
    best = (-1, None)
    for i, j in itertools.combinations(range(12), 2):
        D = np.sqrt(sum((X[i, l] - X[j, l]) ** 2 for l in range(5)))
        E = np.sqrt(sum((Y[i, m] - Y[j, m]) ** 2 for m in range(3)))
        v = abs(E / D - 1)
        if v > best[0]:
            best = (v, (i, j), 1 if E > D else -1)
    c = certificate.certify(X, Y)
    assert abs(c["max"] - best[0]) < 1e-14
    assert (c["i"], c["j"]) == best[1]
    assert c["side"] == best[2]


def test_certificate_two_points_closed_form():
    X = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0]])
    Y = np.array([[1.0], [7.0]])
    c = certificate.certify(X, Y)
    assert c["max"] == pytest.approx(abs(6.0 / 5.0 - 1), abs=1e-15)
    assert (c["i"], c["j"], c["side"]) == (0, 1, 1)
    Y2 = np.array([[0.0], [2.5]])
    c2 = certificate.certify(X, Y2)
    assert c2["max"] == pytest.approx(0.5, abs=1e-15) and c2["side"] == -1


def test_certificate_invariances():
    """delta(Pi) is unchanged by X -> a X + c (Pi linear) and by permuting
    points; the argmax moves with the permutation."""
    X = gen.gaussian(60, 14, seed=17).astype(np.float64)
    Pi = np.random.default_rng(7).standard_normal((5, 14))
    c0 = certificate.certify(X, X @ Pi.T)
    X2 = 2.5 * X + np.arange(14)
    c1 = certificate.certify(X2, X2 @ Pi.T)
    assert abs(c0["max"] - c1["max"]) < 1e-12
    perm = np.random.default_rng(8).permutation(60)
    Xp = X[perm]
    c2 = certificate.certify(Xp, Xp @ Pi.T)
    assert abs(c0["max"] - c2["max"]) < 1e-13
    inv = np.argsort(perm)
    assert {inv[c0["i"]], inv[c0["j"]]} == {c2["i"], c2["j"]}


def test_certificate_skips_identical_points():
    X = gen.with_duplicates(gen.gaussian(30, 6, seed=18), 5).astype(np.float64)
    Y = X @ np.random.default_rng(9).standard_normal((6, 2))
    c = certificate.certify(X, Y)
    D = pdist(X)
    assert c["n_zero"] == int((D == 0).sum()) > 0
    best, _ = _pdist_certificate(X, Y)
    assert abs(c["max"] - best) < 1e-14
    same = np.vstack([X[0]] * 5)
    c0 = certificate.certify(same, same[:, :2])
    assert c0["max"] == 0.0 and c0["n_zero"] == 10 and c0["i"] == -1


def test_certificate_row_blocks_and_pair_list():
    X = gen.gaussian(40, 8, seed=19).astype(np.float64)
    Y = X @ np.random.default_rng(4).standard_normal((8, 3))
    full = certificate.certify(X, Y)
    parts = [certificate.certify(X, Y, rows=(a, a + 10)) for a in range(0, 40, 10)]
    assert max(p["max"] for p in parts) == full["max"]
    assert sum(p["n_pairs"] for p in parts) == full["n_pairs"]
    I = np.array([full["i"], 0, 3]); J = np.array([full["j"], 1, 39])
    v, side = certificate.pair_distortions(X, Y, I, J)
    assert v[0] == full["max"] and side[0] == full["side"]


def test_cross_certificate_is_a_sample_of_the_pairs():
    """Pairs between two index lists (i < j): all rows against all rows is
    the full certificate, bit for bit; a row block against all rows is the
    row-block certificate; two disjoint blocks are brute force over their
    cross pairs; one row against every row (both directions) holds every
    pair of that row."""
    X = gen.gaussian(50, 9, seed=23).astype(np.float64)
    X[31] = X[7]
    Y = X @ np.random.default_rng(6).standard_normal((9, 4))
    allr = np.arange(50)
    full = certificate.certify(X, Y)
    cross = certificate.certify_cross(X, Y, allr, allr)
    assert cross == full
    blk = certificate.certify(X, Y, rows=(10, 20))
    assert certificate.certify_cross(X, Y, np.arange(10, 20), allr) == blk
    A, B = np.arange(5, 15), np.arange(30, 42)
    c = certificate.certify_cross(X, Y, A, B)
    best = max((abs(np.linalg.norm(Y[i] - Y[j]) / np.linalg.norm(X[i] - X[j]) - 1), i, j)
               for i in A for j in B if np.any(X[i] != X[j]))
    assert abs(c["max"] - best[0]) < 1e-14 and (c["i"], c["j"]) == best[1:]
    assert c["n_pairs"] == len(A) * len(B)
    assert certificate.certify_cross(X, Y, B, A)["n_pairs"] == 0
    row = 7
    lo = certificate.certify_cross(X, Y, allr, [row])
    hi = certificate.certify_cross(X, Y, [row], allr)
    assert lo["n_pairs"] + hi["n_pairs"] == 49 and lo["n_zero"] + hi["n_zero"] == 1
    v, _ = certificate.pair_distortions(X, Y, np.minimum(row, allr[allr != row]), np.maximum(row, allr[allr != row]))
    assert max(lo["max"], hi["max"]) == v.max()


# ---------------------------------------------------------------- search
def test_pca_search_equals_linear_scan():
    """For PCA alone ||P_s v|| grows with s, so the distortion is monotone in r
    and bisection must return the smallest r meeting eps."""
    X = gen.low_rank_pixels(n=100, d=30, rank=6, noise=0.08, seed=20)
    _, _, _, Vt = pca.pca(X)
    for eps in (0.05, 0.2, 0.5):
        f = search.fit(X, eps, 1, family="pca")
        deltas = [search.distortion_of_map(X, embedding.pca_map(Vt, r))["max"] for r in range(1, 31)]
        assert all(a >= b - 1e-12 for a, b in zip(deltas, deltas[1:]))
        first = next(r for r, dl in zip(range(1, 31), deltas) if dl <= eps)
        assert f["r"] == first


def test_adagio_search_contract():
    """r* meets eps; every probe below the final lo failed or was r* itself."""
    X = gen.low_rank_pixels(n=150, d=48, rank=6, seed=21)
    f = search.fit(X, 0.15, 5388)
    assert f["cert"]["max"] <= 0.15
    fails = [r for r, v in f["probes"] if v > 0.15]
    assert all(r < f["r"] for r in fails)
    assert int(np.floor(np.log2(48))) <= len(f["probes"]) <= int(np.ceil(np.log2(48)))


def test_jl_cannot_reduce_at_small_eps():
    """Sec. 4.3: for small delta JL alone needs the ambient dimension."""
    X = gen.low_rank_pixels(n=120, d=64, rank=6, seed=22)
    f = search.fit(X, 0.05, 5388, family="jl")
    assert f["r"] == 64
