"""Sketch features of the learned search (oracle, FP64).  Test
infrastructure only.

Not part of the paper.  G = Omega Xc with Xc the centred cloud and Omega a
m x n matrix of +-1/sqrt(m) signs (m = 128): entry (a, i) is + when bit 63 of
SplitMix64 output number a * 2^32 + i + 1 of the generator seeded with
seed ^ 0xD1B54A32D192ED03 is 0.  With lam the eigenvalues of G G^T in
decreasing order and sigma = sqrt(max(lam, 0)):
  f[i] = ln(sigma_i / ||sigma|| + 1e-6) / 4   (i < 64)
  f[64] = ln(n) / 10, f[65] = ln(d) / 10, f[66] = 5 eps, f[67..79] = 0.
"""
import numpy as np

from .jl_signs import splitmix64_output

SKETCH_ROWS = 128
STREAM = 0xD1B54A32D192ED03


def sketch_signs(seed, m, n):
    a = np.arange(m, dtype=np.uint64)[:, None]
    i = np.arange(n, dtype=np.uint64)[None, :]
    z = splitmix64_output(np.uint64(seed) ^ np.uint64(STREAM), ((a << np.uint64(32)) | i) + np.uint64(1))
    return np.where((z >> np.uint64(63)) == 0, 1.0, -1.0) / np.sqrt(m)


def sketch_features(X, eps, seed, m=SKETCH_ROWS):
    X = np.asarray(X, np.float64)
    n, d = X.shape
    Xc = X - X.mean(axis=0)
    G = sketch_signs(seed, m, n) @ Xc
    lam = np.sort(np.linalg.eigvalsh(G @ G.T))[::-1]
    lam = np.maximum(lam, 0.0)
    norm = np.sqrt(lam.sum()) or 1.0
    f = np.zeros(80)
    f[:64] = np.log(np.sqrt(lam[:64]) / norm + 1e-6) / 4.0
    f[64] = np.log(n) / 10.0
    f[65] = np.log(d) / 10.0
    f[66] = 5.0 * eps
    return f
