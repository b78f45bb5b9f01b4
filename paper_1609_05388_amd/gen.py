"""Seeded synthetic point clouds.

This module only draws inputs; it holds none of the method's arithmetic.  All
arrays are drawn in FP64 with numpy's PCG64 ``default_rng`` in the fixed order
written in each function and then cast to FP32; the FP32 array is the
canonical input for both the library and its checker.

The paper's datasets (MNIST, UCR, UCI, ZuBuD) are not available; these clouds
stand in for them with the same shapes and the structure that matters to a
data-aware embedding: a low intrinsic rank with a noise floor, pixel values in
[0, 1], and (for the MNIST-shaped cloud) a fixed blank border of 549 of 784
pixels.
"""
import numpy as np

DATA_SEED = 1609
JL_SEED = 5388


def _orthonormal(rng, d, q):
    """d x q matrix with orthonormal columns (QR of a Gaussian matrix)."""
    return np.linalg.qr(rng.standard_normal((d, q)))[0]


def low_rank_pixels(n=2000, d=784, rank=40, noise=0.05, seed=DATA_SEED):
    """clip(U z + noise * e, 0, 1) with U a random d x rank orthonormal basis,
    z ~ N(0, 1)^rank and e ~ N(0, 1)^d per point.
    Draw order: U, Z (n x rank), E (n x d)."""
    rng = np.random.default_rng(seed)
    U = _orthonormal(rng, d, rank)
    Z = rng.standard_normal((n, rank))
    E = rng.standard_normal((n, d))
    return np.clip(Z @ U.T + noise * E, 0.0, 1.0).astype(np.float32)


def mnist_shaped(n=60000, d=784, rank=50, classes=10, class_std=0.3, active=235,
                 seed=DATA_SEED):
    """MNIST-shaped pixels in [0, 1]: m * clip(Zc B^T, 0, 1) where B is a random
    d x rank orthonormal basis, Zc = A[c] + class_std * N(0, 1) with A the
    classes x rank class means, c uniform class labels, and m a fixed mask with
    ``active`` ones (70% of 784 pixels are always zero, like a blank border).
    Draw order: B, A, c, noise (n x rank), mask permutation."""
    rng = np.random.default_rng(seed)
    B = _orthonormal(rng, d, rank)
    A = rng.standard_normal((classes, rank))
    c = rng.integers(0, classes, size=n)
    Zc = A[c] + class_std * rng.standard_normal((n, rank))
    mask = np.zeros(d)
    mask[rng.permutation(d)[:active]] = 1.0
    X = np.clip(Zc @ B.T, 0.0, 1.0) * mask
    return X.astype(np.float32)


def power_law(n, d, rank, alpha, noise=0.01, seed=DATA_SEED, chunk=8192):
    """X = (Z * sigma) U^T + noise * E with sigma_i = i^-alpha over ``rank``
    directions.  Draw order: U (d x rank), Z (n x rank), then E in row chunks
    of ``chunk`` rows, each chunk from its own spawned child generator."""
    rng = np.random.default_rng(seed)
    U = _orthonormal(rng, d, rank)
    Z = rng.standard_normal((n, rank))
    sigma = np.arange(1, rank + 1, dtype=np.float64) ** (-float(alpha))
    children = np.random.SeedSequence(seed).spawn((n + chunk - 1) // chunk)
    X = np.empty((n, d), dtype=np.float32)
    for t, ss in enumerate(children):
        a, b = t * chunk, min(n, (t + 1) * chunk)
        E = np.random.default_rng(ss).standard_normal((b - a, d))
        X[a:b] = ((Z[a:b] * sigma) @ U.T + noise * E).astype(np.float32)
    return X


def gaussian(n, d, seed=DATA_SEED, scale=1.0, offset=0.0):
    """Plain N(offset, scale^2) points (ragged-shape and edge-case tests)."""
    rng = np.random.default_rng(seed)
    return (offset + scale * rng.standard_normal((n, d))).astype(np.float32)


def exact_rank(n, d, q, seed=DATA_SEED):
    """Points on a q-dimensional affine subspace (no noise)."""
    rng = np.random.default_rng(seed)
    U = _orthonormal(rng, d, q)
    Z = rng.standard_normal((n, q))
    c = rng.standard_normal(d)
    return (Z @ U.T + c).astype(np.float32)


def with_duplicates(X, n_dup, seed=DATA_SEED):
    """Copy ``n_dup`` randomly chosen rows over other rows (identical points)."""
    rng = np.random.default_rng(seed + 1)
    X = X.copy()
    n = X.shape[0]
    src = rng.integers(0, n, size=n_dup)
    dst = rng.integers(0, n, size=n_dup)
    X[dst] = X[src]
    return X


def instance_params(index, held_out=False):
    """Parameters of one learned-form training instance: n ~ U{1000..20000},
    d ~ U{128, 256, 784, 2048}, alpha ~ U[0.5, 2], rank ~ U{10..200} capped at
    d, eps ~ U[0.05, 0.3].  Seeds 10000 + t (training) and 90000 + t (held out)."""
    seed = (90000 if held_out else 10000) + int(index)
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1000, 20001))
    d = int(rng.choice([128, 256, 784, 2048]))
    alpha = float(rng.uniform(0.5, 2.0))
    rank = int(min(rng.integers(10, 201), d))
    eps = float(rng.uniform(0.05, 0.3))
    return {"seed": seed, "n": n, "d": d, "alpha": alpha, "rank": rank, "eps": eps}


def sift_shaped(buildings=201, photos=4, per_photo=500, per_query=100, proto=500, clutter=3000,
                latent=48, own=0.22, noise=0.065, seed=DATA_SEED):
    """SIFT-shaped descriptors of a building-retrieval workload (the image
    retrieval experiment of Sec. 4.6's nearest-neighbour queries): ``buildings``
    objects, ``photos`` database photos of ``per_photo`` descriptors each and
    one query photo of ``per_query`` descriptors per object, all in R^128.

    A descriptor is a prototype seen with noise.  Prototypes are
    sift(relu(A z)) with z ~ N(0, 1)^latent and A a 128 x latent Gaussian
    matrix whose column j is scaled by (j + 1)^-0.7, so that most variance
    sits in a few dozen directions as for real SIFT; sift(v) is SIFT's own
    normalisation: unit length, entries clipped at 0.2, unit length again.
    Each object owns ``proto`` prototypes; a pool of ``clutter`` prototypes
    is shared by all objects.  A photo draws a fraction ``own`` of its
    descriptors from its object's prototypes and the rest from the pool (both
    uniformly), and each descriptor is round(512 sift(relu(p + noise e))),
    e ~ N(0, 1)^128, as integers in FP32.

    Returns (D, d_label, Q, q_image): the database (buildings * photos *
    per_photo x 128, object by object, photo by photo), the object of each
    database row, the queries (buildings * per_query x 128, object by
    object) and the object of each query row.
    Draw order: A, object prototypes, pool, then per object: database photos
    (choices, pool choices, noise) and the query photo (same)."""
    rng = np.random.default_rng(seed)
    m = 128
    A = rng.standard_normal((m, latent)) * (np.arange(1, latent + 1, dtype=np.float64) ** -0.7)

    def sift(v):
        v = v / np.maximum(np.linalg.norm(v, axis=-1, keepdims=True), 1e-12)
        v = np.minimum(v, 0.2)
        return v / np.maximum(np.linalg.norm(v, axis=-1, keepdims=True), 1e-12)

    def protos(cnt):
        return sift(np.maximum(rng.standard_normal((cnt, latent)) @ A.T, 0.0))

    P = protos(buildings * proto).reshape(buildings, proto, m)
    pool = protos(clutter)

    def photo(b, cnt):
        n_own = int(round(own * cnt))
        src = np.concatenate([P[b][rng.integers(0, proto, n_own)], pool[rng.integers(0, clutter, cnt - n_own)]])
        e = rng.standard_normal((cnt, m))
        return np.round(512.0 * sift(np.maximum(src + noise * e, 0.0)))

    D, Q = [], []
    for b in range(buildings):
        for _ in range(photos):
            D.append(photo(b, per_photo))
        Q.append(photo(b, per_query))
    D = np.concatenate(D).astype(np.float32)
    Q = np.concatenate(Q).astype(np.float32)
    d_label = np.repeat(np.arange(buildings, dtype=np.int32), photos * per_photo)
    q_image = np.repeat(np.arange(buildings, dtype=np.int32), per_query)
    return D, d_label, Q, q_image
