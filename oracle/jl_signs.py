"""Johnson-Lindenstrauss sign matrix S (oracle).  Test infrastructure only.

Lemma 1 and Algorithm 1 ask for a k x d matrix whose entries are chosen
uniformly and independently from {-1/sqrt(k), +1/sqrt(k)}.  The paper does not
name a generator, so (reading) the entries come from a fixed, infinite sign
matrix B in {-1,+1}^(inf x d):

    b[a, l] = +1 if bit 63 of SplitMix64(seed) output number c + 1 is 0,
              -1 otherwise,      with counter c = a * 2**32 + l,

and S_k = B[:k, :] / sqrt(k).  Rows are therefore nested across k.

SplitMix64 is the generator of Steele, Lea and Flood ("Fast splittable
pseudorandom number generators", OOPSLA 2014): the state advances by the odd
constant 0x9E3779B97F4A7C15 and each output is the state passed through the
published 64-bit finaliser (xor-shift 30, multiply, xor-shift 27, multiply,
xor-shift 31).  Output number t of a generator seeded with `seed` is
finaliser(seed + t * 0x9E3779B97F4A7C15 mod 2**64), t = 1, 2, ...

This module is written independently of the GPU library's generator; the two
agree only because both follow the published definition.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_output(seed, t):
    """Output number ``t`` (t >= 1, array) of SplitMix64 seeded with ``seed``."""
    t = np.asarray(t, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + t * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def sign_matrix(seed, k, d):
    """The first k rows of B as float64 +-1 values (shape k x d)."""
    if k == 0:
        return np.zeros((0, d))
    a = np.arange(k, dtype=np.uint64)[:, None]
    l = np.arange(d, dtype=np.uint64)[None, :]
    counter = (a << np.uint64(32)) | l
    z = splitmix64_output(seed, counter + np.uint64(1))
    top = (z >> np.uint64(63)).astype(np.int64)
    return np.where(top == 0, 1.0, -1.0)


def jl_matrix(seed, k, d):
    """S_k = B[:k] / sqrt(k): Lemma 1's +-1/sqrt(k) matrix (FP64)."""
    if k == 0:
        return np.zeros((0, d))
    return sign_matrix(seed, k, d) / np.sqrt(k)
