"""FP64 reference of the learned form's predictor (oracle).  Test
infrastructure only.

Not part of the paper: the learned form predicts ln(r / d) for the
target-dimension search.  Network: x (80 inputs, 67 used) -> relu(W1 x + b1)
-> relu(W2 . + b2) -> relu(W3 . + b3) -> w4 . + b4.  Loss: pinball loss at level
tau of u = y - out, mean over the batch: max(tau u, (tau - 1) u).  The
gradient is written out by the chain rule; the pins check it against central
finite differences.

Parameters use the library's flat layout: W1[256][80], b1[256], W2[256][256],
b2[256], W3[256][256], b3[256], w4[256], b4, 3 padding values.
"""
import numpy as np

IN_PAD, HID = 80, 256


def layout():
    off = {}
    o = 0
    for name, size in (("W1", HID * IN_PAD), ("b1", HID), ("W2", HID * HID), ("b2", HID),
                       ("W3", HID * HID), ("b3", HID), ("w4", HID), ("b4", 1)):
        off[name] = (o, size)
        o += size
    return off, o + 3


def unpack(p):
    off, _ = layout()
    g = {k: p[o:o + s] for k, (o, s) in off.items()}
    return (g["W1"].reshape(HID, IN_PAD), g["b1"], g["W2"].reshape(HID, HID), g["b2"],
            g["W3"].reshape(HID, HID), g["b3"], g["w4"], g["b4"][0])


def forward(p, X, round_act=None):
    """round_act (optional): applied to the hidden activations A1 and A2 where
    they become the next layer's operand, so that a reduced-precision network
    can be followed with its own ReLU decisions (the rest stays FP64)."""
    W1, b1, W2, b2, W3, b3, w4, b4 = unpack(np.asarray(p, np.float64))
    X = np.asarray(X, np.float64)
    r = round_act or (lambda a: a)
    Z1 = X @ W1.T + b1
    A1 = r(np.maximum(Z1, 0.0))
    Z2 = A1 @ W2.T + b2
    A2 = r(np.maximum(Z2, 0.0))
    Z3 = A2 @ W3.T + b3
    A3 = np.maximum(Z3, 0.0)
    out = A3 @ w4 + b4
    return out, (X, Z1, A1, Z2, A2, Z3, A3)


def loss(p, X, y, tau):
    out, _ = forward(p, X)
    u = np.asarray(y, np.float64) - out
    return np.mean(np.maximum(tau * u, (tau - 1.0) * u))


def grad(p, X, y, tau, round_act=None):
    """Loss and gradient by the chain rule (subgradient -tau at u = 0+)."""
    p = np.asarray(p, np.float64)
    W1, b1, W2, b2, W3, b3, w4, b4 = unpack(p)
    out, (X, Z1, A1, Z2, A2, Z3, A3) = forward(p, X, round_act)
    B = X.shape[0]
    u = np.asarray(y, np.float64) - out
    L = np.mean(np.maximum(tau * u, (tau - 1.0) * u))
    g = np.where(u > 0, -tau, 1.0 - tau) / B           # dL/dout
    gw4 = A3.T @ g
    gb4 = g.sum()
    dZ3 = np.outer(g, w4) * (Z3 > 0)
    gW3 = dZ3.T @ A2
    gb3 = dZ3.sum(0)
    dZ2 = (dZ3 @ W3) * (Z2 > 0)
    gW2 = dZ2.T @ A1
    gb2 = dZ2.sum(0)
    dZ1 = (dZ2 @ W2) * (Z1 > 0)
    gW1 = dZ1.T @ X
    gb1 = dZ1.sum(0)
    _, total = layout()
    G = np.zeros(total)
    off, _ = layout()
    for name, val in (("W1", gW1), ("b1", gb1), ("W2", gW2), ("b2", gb2), ("W3", gW3), ("b3", gb3),
                      ("w4", gw4), ("b4", np.array([gb4]))):
        o, s = off[name]
        G[o:o + s] = np.ravel(val)
    return L, G
