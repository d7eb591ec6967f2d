"""Oracle of the learned phase schedule (test infrastructure only: imported by
tests, never by the library or the benchmark's product path).

The schedule's value network is a plain multilayer perceptron
    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  q = W3 h2 + b3
with x in R^F, h1, h2 in R^H, q in R^K (one output per phase action).  It is
fitted by regression of the taken action only: for samples (x_i, a_i, y_i),
    L = (1/N) sum_i (q_i[a_i] - y_i)^2,
so the gradient reaches only the output of the action that was taken.  The
derivative of relu at 0 is taken as 0.  Parameters are one flat vector in the
order W1 (H x F, row-major), b1, W2 (H x H), b2, W3 (K x H), b3.

Everything here is fp64 numpy.  Pins (tests/test_oracle_mlp.py): central
finite differences of L, and the closed form of linear least squares when the
hidden layers pass the input through unchanged.

The phase features (`phase_features`) follow the definitions stated in
include/mf.h for mf_set_policy: the quantities of the state right after a
global relabel, scaled to roughly [0, 1].
"""
from __future__ import annotations

import numpy as np

F, H, K = 16, 32, 8


def n_params(f: int = F, h: int = H, k: int = K) -> int:
    return h * f + h + h * h + h + k * h + k


def unpack(theta, f: int = F, h: int = H, k: int = K):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (n_params(f, h, k),)
    o = 0
    W1 = theta[o:o + h * f].reshape(h, f); o += h * f
    b1 = theta[o:o + h]; o += h
    W2 = theta[o:o + h * h].reshape(h, h); o += h * h
    b2 = theta[o:o + h]; o += h
    W3 = theta[o:o + k * h].reshape(k, h); o += k * h
    b3 = theta[o:o + k]; o += k
    return W1, b1, W2, b2, W3, b3


def forward(theta, X):
    """q (N x K) for inputs X (N x F)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    return h2 @ W3.T + b3


def loss(theta, X, a, y) -> float:
    q = forward(theta, X)
    a = np.asarray(a, dtype=np.int64)
    r = q[np.arange(q.shape[0]), a] - np.asarray(y, dtype=np.float64)
    return float(np.mean(r * r))


def loss_and_grad(theta, X, a, y):
    """L and dL/dtheta by the chain rule, layer by layer."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    a = np.asarray(a, dtype=np.int64)
    y = np.asarray(y, dtype=np.float64)
    N = X.shape[0]
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    q = h2 @ W3.T + b3
    rows = np.arange(N)
    r = q[rows, a] - y
    L = float(np.mean(r * r))
    dq = np.zeros_like(q)
    dq[rows, a] = 2.0 * r / N
    gW3 = dq.T @ h2
    gb3 = dq.sum(axis=0)
    dz2 = (dq @ W3) * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, g


def adam_step(theta, g, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) with bias correction; t counts
    from 1.  Returns the new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def phase_features(n: int, e: np.ndarray, h: np.ndarray, s: int, t: int, levels: int,
                   prev_pushes: int, prev_relabels: int, phase: int, batch_fraction: float):
    """The 16 features of a phase from the state right after its global
    relabel: heights h (|V| = unreached) and excesses e.  Computed in float32
    where the device computes in float32."""
    f32 = np.float32
    e = np.asarray(e, dtype=np.int64)
    h = np.asarray(h, dtype=np.int64)
    idx = np.arange(n)
    active = (e > 0) & (h < n) & (idx != s) & (idx != t)
    cnt = int(active.sum())
    esum = int(e[active].sum())
    out = np.zeros(16, dtype=np.float32)
    out[0] = f32(np.log2(f32(1 + cnt))) / f32(24)
    out[1] = f32(np.log2(f32(1 + esum))) / f32(40)
    if cnt:
        lg = np.floor(np.log2(e[active].astype(np.float64))).astype(np.int64)  # exact for int64 < 2^53
        bins = np.minimum(lg >> 2, 7)
        hist = np.bincount(bins, minlength=8)
        out[2:10] = (hist.astype(np.float32) / f32(cnt)).astype(np.float32)
    out[10] = f32(np.log2(f32(1 + levels))) / f32(12)
    out[11] = f32(int((h < n).sum())) / f32(n)
    out[12] = f32(np.log2(f32(1 + prev_pushes))) / f32(32)
    out[13] = f32(np.log2(f32(1 + prev_relabels))) / f32(32)
    out[14] = f32(np.log2(f32(1 + phase))) / f32(8)
    out[15] = f32(batch_fraction)
    return out
