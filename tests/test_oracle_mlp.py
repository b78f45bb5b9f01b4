"""Pins of the learned form's FP64 oracle: the chain-rule gradient of the
pinball-loss MLP against central finite differences, and the sketch-feature
definition against its own pieces."""
import numpy as np
import pytest

from oracle import mlp, sketch
from paper_1609_05388_amd import gen


def random_params(seed):
    rng = np.random.default_rng(seed)
    _, total = mlp.layout()
    p = rng.normal(0, 0.08, total)
    off, _ = mlp.layout()
    o, s = off["W1"]
    W1 = p[o:o + s].reshape(256, 80)
    W1[:, 67:] = 0.0
    return p


def batch(seed, B=16):
    rng = np.random.default_rng(seed)
    X = np.zeros((B, 80))
    X[:, :67] = rng.normal(0, 1, (B, 67))
    y = rng.normal(-1.5, 0.5, B)
    return X, y


def test_gradient_matches_central_differences():
    """The network and loss are piecewise linear: central differences with a
    small step reproduce the chain rule exactly away from kinks."""
    p = random_params(1)
    X, y = batch(2)
    L, G = mlp.grad(p, X, y, 0.9)
    assert abs(L - mlp.loss(p, X, y, 0.9)) < 1e-15
    rng = np.random.default_rng(3)
    off, total = mlp.layout()
    idx = np.concatenate([rng.choice(total - 3, 300, replace=False), [off["b4"][0]]])
    h = 1e-7
    for k in idx:
        e = np.zeros(total)
        e[k] = h
        fd = (mlp.loss(p + e, X, y, 0.9) - mlp.loss(p - e, X, y, 0.9)) / (2 * h)
        assert abs(fd - G[k]) <= 1e-6 * max(1.0, abs(G[k])), k


def test_pinball_loss_closed_form():
    """With all weights zero the output is b4: L = mean of the pinball terms."""
    _, total = mlp.layout()
    p = np.zeros(total)
    off, _ = mlp.layout()
    p[off["b4"][0]] = 0.5
    X, _ = batch(4, B=4)
    y = np.array([1.5, 0.5, -0.5, 0.0])
    u = y - 0.5
    want = np.mean(np.maximum(0.9 * u, -0.1 * u))
    assert mlp.loss(p, X, y, 0.9) == pytest.approx(want, abs=1e-15)
    L, G = mlp.grad(p, X, y, 0.9)
    assert G[off["b4"][0]] == pytest.approx(np.mean(np.where(u > 0, -0.9, 0.1)), abs=1e-15)


def test_missing_relu_gate_is_caught(monkeypatch):
    """A planted mistake (no ReLU gate on the first layer's backward) fails
    the finite-difference pin."""
    orig = mlp.grad

    def bad(p, X, y, tau):
        p = np.asarray(p, np.float64)
        W1, b1, W2, b2, W3, b3, w4, b4 = mlp.unpack(p)
        out, (X, Z1, A1, Z2, A2, Z3, A3) = mlp.forward(p, X)
        L, G = orig(p, X, y, tau)
        B = X.shape[0]
        u = np.asarray(y) - out
        g = np.where(u > 0, -tau, 1.0 - tau) / B
        dZ3 = np.outer(g, w4) * (Z3 > 0)
        dZ2 = (dZ3 @ W3) * (Z2 > 0)
        dZ1 = dZ2 @ W2                      # gate dropped
        off, _ = mlp.layout()
        o, s = off["W1"]
        G[o:o + s] = (dZ1.T @ X).ravel()
        return L, G

    monkeypatch.setattr(mlp, "grad", bad)
    with pytest.raises(AssertionError):
        test_gradient_matches_central_differences()


def test_sketch_features_definition():
    """Features of a cloud with an exact low-rank structure: the sketch of a
    rank-q centred cloud has exactly q nonzero singular values, so features
    q..63 sit at ln(1e-6)/4; shape and scalar features follow the definition."""
    X = gen.exact_rank(300, 40, 5, seed=7)
    f = sketch.sketch_features(X, 0.1, 5388)
    assert f.shape == (80,)
    assert np.all(f[5:64] < np.log(1e-5) / 4)
    assert np.all(f[:5] > np.log(1e-3) / 4)
    assert f[64] == pytest.approx(np.log(300) / 10) and f[65] == pytest.approx(np.log(40) / 10)
    assert f[66] == pytest.approx(0.5) and np.all(f[67:] == 0)
    # E[Omega^T Omega] = I: sum of sketch eigenvalues ~ ||Xc||_F^2 (JL, 5 sigma)
    Xc = X.astype(np.float64) - X.astype(np.float64).mean(0)
    G = sketch.sketch_signs(5388, 128, 300) @ Xc
    ratio = np.sum(G * G) / np.sum(Xc * Xc)
    assert abs(ratio - 1.0) < 5 * np.sqrt(2.0 / 128)
