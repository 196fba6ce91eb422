"""Per-vertex skeleton scorer: a small MLP, its loss, gradients and Adam
(oracle; test infrastructure only).

Not in the paper: it learns to propose the rows/columns of the pseudo-skeleton
of Sec. 5.3 (eq. Ahat) that BDLR picks by boundary distance.  Network, per
vertex with 8 features x:

    h1 = relu(W1 x + b1)        W1: 64 x 8
    h2 = relu(W2 h1 + b2)       W2: 64 x 64
    z  = w3 . h2 + b3           w3: 64

Loss over N vertices with labels y in {0, 1} (1 = a pivot of that block) and
positive-class weight p (weighted binary cross-entropy on the logit):

    l_i = p y_i softplus(-z_i) + (1 - y_i) softplus(z_i),   L = mean_i l_i

Adam (Kingma & Ba, 2015) with bias correction:

    m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
    theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Pinned in tests: central finite differences of every gradient, the loss at
hand-computed points, and one Adam step worked by hand.
"""
from __future__ import annotations

import numpy as np

NF, H = 8, 64
NAMES = ("W1", "b1", "W2", "b2", "w3", "b3")
SHAPES = {"W1": (H, NF), "b1": (H,), "W2": (H, H), "b2": (H,), "w3": (H,), "b3": (1,)}


def softplus(z):
    """log(1 + exp(z)), computed without overflow."""
    z = np.asarray(z, dtype=np.float64)
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    z = np.asarray(z, dtype=np.float64)
    e = np.exp(-np.abs(z))
    return np.where(z >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def forward(params, X):
    """Logits z (N,) and the activations the backward pass needs."""
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ params["W1"].T + params["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ params["W2"].T + params["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ params["w3"] + params["b3"][0]
    return z, (X, a1, h1, a2, h2)


def loss(params, X, y, pos_weight):
    z, _ = forward(params, X)
    y = np.asarray(y, dtype=np.float64)
    return float(np.mean(pos_weight * y * softplus(-z) + (1.0 - y) * softplus(z)))


def loss_and_grad(params, X, y, pos_weight):
    """Mean loss and its gradient with respect to every parameter."""
    z, (X, a1, h1, a2, h2) = forward(params, X)
    y = np.asarray(y, dtype=np.float64)
    N = z.shape[0]
    L = float(np.mean(pos_weight * y * softplus(-z) + (1.0 - y) * softplus(z)))
    # dl/dz = -p y sigmoid(-z) + (1 - y) sigmoid(z)
    dz = (-pos_weight * y * sigmoid(-z) + (1.0 - y) * sigmoid(z)) / N
    g = {"w3": h2.T @ dz, "b3": np.array([dz.sum()])}
    dh2 = np.outer(dz, params["w3"])
    da2 = dh2 * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ params["W2"]
    da1 = dh1 * (a1 > 0)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(axis=0)
    return L, g


def adam_step(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (params, m, v)."""
    P, M, V = {}, {}, {}
    for k in NAMES:
        M[k] = beta1 * m[k] + (1.0 - beta1) * grads[k]
        V[k] = beta2 * v[k] + (1.0 - beta2) * grads[k] ** 2
        mh = M[k] / (1.0 - beta1 ** t)
        vh = V[k] / (1.0 - beta2 ** t)
        P[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return P, M, V


def random_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return {k: rng.normal(0.0, scale, SHAPES[k]) for k in NAMES}


def round_bf16(a):
    """Round float64 values to bfloat16 (through float32, nearest-even)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    out = u.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(f), f, out).astype(np.float64)
