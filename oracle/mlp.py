"""Learned start network in FP64 (test infrastructure only).

Not part of the paper: the paper starts from back-propagation
(Eq. backpropagation). This is the network that proposes start rows from a
row's intensities: input 4N = K N features I_p / mean(I_p), two hidden
layers of width H with GELU (erf form), output 2N reals read as the
complex start u = o[:N] + j o[N:].

Loss per row: ||u||^2 + ||u*||^2 - 2 |u*^H u| with the target
u* = t / s, s = sqrt(sum(I_p) / (K N)); the loss is invariant to the row's
unknown phase (Sec. 2.3, Eq. phaseoffset) and its packed gradient
(d/dRe + j d/dIm, the paper's convention of Eq. derivative) is
2 (u - e^{j arg(u*^H u)} u*). Inference rescales u to norm s (Parseval,
A^H A = K N I). Optimiser: Adam.
"""
from __future__ import annotations

import math

import numpy as np

_erf = np.vectorize(math.erf)


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + _erf(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def features(I: np.ndarray) -> np.ndarray:
    """[B, K, N] intensities -> [B, K N] features I / mean(I_p)."""
    X = I.reshape(I.shape[0], -1)
    m = X.mean(axis=1, keepdims=True)
    return X / np.where(m > 0, m, 1.0)


def row_scale(I: np.ndarray, K: int, N: int) -> np.ndarray:
    return np.sqrt(I.reshape(I.shape[0], -1).sum(axis=1) / (K * N))


def init_params(n_in: int, hidden: int, n_out: int, g: np.random.Generator):
    """He-style normal init scaled by 1/sqrt(fan_in); zero biases."""
    return {
        "W1": g.standard_normal((n_in, hidden)) / math.sqrt(n_in),
        "b1": np.zeros(hidden),
        "W2": g.standard_normal((hidden, hidden)) / math.sqrt(hidden),
        "b2": np.zeros(hidden),
        "W3": g.standard_normal((hidden, n_out)) / math.sqrt(hidden),
        "b3": np.zeros(n_out),
    }


def forward(p, X):
    a1 = X @ p["W1"] + p["b1"]
    h1 = gelu(a1)
    a2 = h1 @ p["W2"] + p["b2"]
    h2 = gelu(a2)
    o = h2 @ p["W3"] + p["b3"]
    return o, (X, a1, h1, a2, h2)


def split_complex(o):
    n = o.shape[1] // 2
    return o[:, :n] + 1j * o[:, n:]


def loss_and_dout(o, target):
    """Mean over rows of ||u||^2 + ||u*||^2 - 2|u*^H u| and its gradient
    with respect to the real outputs o (d/do = [Re, Im] of the packed
    gradient 2(u - e^{j arg c} u*), divided by the batch)."""
    u = split_complex(o)
    c = np.sum(np.conj(target) * u, axis=1)
    L = np.sum(np.abs(u) ** 2, 1) + np.sum(np.abs(target) ** 2, 1) - 2 * np.abs(c)
    ph = np.where(np.abs(c) > 0, c / np.where(np.abs(c) > 0, np.abs(c), 1.0), 1.0)
    gp = 2.0 * (u - ph[:, None] * target) / o.shape[0]
    return float(L.mean()), np.concatenate([gp.real, gp.imag], axis=1)


def backward(p, cache, dout):
    X, a1, h1, a2, h2 = cache
    grads = {}
    grads["W3"] = h2.T @ dout
    grads["b3"] = dout.sum(0)
    dh2 = dout @ p["W3"].T
    da2 = dh2 * gelu_grad(a2)
    grads["W2"] = h1.T @ da2
    grads["b2"] = da2.sum(0)
    dh1 = da2 @ p["W2"].T
    da1 = dh1 * gelu_grad(a1)
    grads["W1"] = X.T @ da1
    grads["b1"] = da1.sum(0)
    return grads


def adam_step(p, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1 - b1) * grads[k]
        v[...] = b2 * v + (1 - b2) * grads[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def predict_start(p, I, K, N):
    """Start rows from the network: u rescaled to ||t||^2 = sum(I)/(K N)."""
    o, _ = forward(p, features(I))
    u = split_complex(o)
    n = np.linalg.norm(u, axis=1)
    return u / np.where(n > 0, n, 1.0)[:, None] * row_scale(I, K, N)[:, None]
