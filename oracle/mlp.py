"""FP64 reference of the rank predictor: a multilayer perceptron with three
hidden ReLU layers of 64 units, its loss, gradient and Adam step.

TEST INFRASTRUCTURE ONLY (see the package header).

The predictor maps six box features to the ID rank of the box (the larger of
its two halves' ranks).  The paper motivates predetermining ranks so that
work can be sized before the factorisation (Section 4.3, the discussion of
parallel efficiency with fixed ranks); the network, its features and loss
are this project's design:

  features  f = (k_out d, k_in d, mean|kappa| d, max|kappa| d, level, log10 tol)
            with d the box diameter (twice the largest distance of its nodes
            from the bounding-box midpoint), kappa the curvature at its nodes,
            level the box's level in its boundary's tree;
  input     x = (f - mu) / sigma  (feature normalisation stored with the weights)
  network   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), h3 = relu(W3 h2 + b3),
            yhat = W4 h3 + b4   (a prediction of log(rank))
  loss      L = (1/n) sum_s c_s r_s^2,  r_s = yhat_s - log(rank_s),
            c_s = alpha if r_s < 0 (under-prediction, which costs a fallback)
            else 1.

Parameters are one flat float vector in the order W1 (64 x 6, row-major:
W[o, i] at o * nin + i), b1, W2 (64 x 64), b2, W3 (64 x 64), b3, W4 (1 x 64),
b4: 8833 values.  Adam follows Kingma & Ba (2015): m = b1 m + (1 - b1) g,
v = b2 v + (1 - b2) g^2, p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""

from __future__ import annotations

import numpy as np

LAYERS = [(6, 64), (64, 64), (64, 64), (64, 1)]
N_FEATURES = 6


def n_params() -> int:
    return sum(i * o + o for i, o in LAYERS)


def unpack(p: np.ndarray):
    """Flat parameter vector -> [(W, b), ...] views (W is out x in)."""
    out, k = [], 0
    for i, o in LAYERS:
        W = p[k:k + i * o].reshape(o, i)
        k += i * o
        b = p[k:k + o]
        k += o
        out.append((W, b))
    assert k == p.size
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in LAYERS:
        parts.append(rng.standard_normal(i * o) * np.sqrt(2.0 / i))
        parts.append(np.zeros(o))
    return np.concatenate(parts)


def forward(p: np.ndarray, x: np.ndarray):
    """x: (n, 6) normalised inputs.  Returns yhat (n,) and the activations
    [x, h1, h2, h3] (the inputs of the four layers)."""
    acts = [np.asarray(x, dtype=np.float64)]
    layers = unpack(np.asarray(p, dtype=np.float64))
    h = acts[0]
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        if li < len(layers) - 1:
            h = np.maximum(z, 0.0)
            acts.append(h)
        else:
            h = z
    return h[:, 0], acts


def loss_and_grad(p: np.ndarray, x: np.ndarray, rank: np.ndarray, alpha: float):
    """Loss L and its gradient dL/dp (flat, same layout as p)."""
    yhat, acts = forward(p, x)
    t = np.log(np.asarray(rank, dtype=np.float64))
    r = yhat - t
    c = np.where(r < 0.0, alpha, 1.0)
    n = x.shape[0]
    L = float(np.sum(c * r * r) / n)
    dz = (2.0 / n) * c * r  # dL/dyhat
    dz = dz[:, None]
    layers = unpack(np.asarray(p, dtype=np.float64))
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        a = acts[li]
        grads[li] = (dz.T @ a, dz.sum(axis=0))
        if li > 0:
            da = dz @ W
            dz = da * (acts[li] > 0.0)
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return L, flat


def adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (t counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def normalisation(feat: np.ndarray):
    """Per-feature mean and standard deviation (sigma of a constant feature is 1)."""
    mu = feat.mean(axis=0)
    sd = feat.std(axis=0)
    sd = np.where(sd > 0, sd, 1.0)
    return mu, sd


def box_features(x: np.ndarray, kappa: np.ndarray, lo: int, hi: int, k_out: float, k_in: float, level: int,
                 tol: float) -> np.ndarray:
    """The six features of the box holding nodes lo..hi-1 of one boundary
    (x: (N, 2) nodes, kappa: (N,) curvature)."""
    pts = x[lo:hi]
    c = 0.5 * (pts.min(axis=0) + pts.max(axis=0))
    d = 2.0 * float(np.sqrt(((pts - c) ** 2).sum(axis=1)).max())
    ak = np.abs(kappa[lo:hi])
    return np.array([k_out * d, k_in * d, ak.mean() * d, ak.max() * d, float(level), np.log10(tol)])
