"""Pins of three oracle functions (CPU): the L-BFGS initial scaling
H0 = (s^T y / y^T y) I of the two-loop recursion (Sec. 2.2, Alg. 1, with
the L-BFGS of Nocedal & Wright Alg. 7.4 the paper cites), the truncated
spectral weights, and the FP64 acceptance residual's normalisation. Each
test also shows that a plausible mistake (inverted scaling, a mean over all
rows, dividing by ||I|| instead of ||I||^2) fails it."""
import json
import os

import numpy as np

from oracle import operators as ops
from oracle import retrieval as rt

GOLD = os.path.join(os.path.dirname(__file__), "golden", "weights_residual_example.json")


def _c(a):
    a = np.asarray(a, dtype=np.float64)
    return a[..., 0] + 1j * a[..., 1]


def _real(v):
    """C^N -> R^{2N}; Re(a^H b) is the standard inner product there."""
    return np.concatenate([v.real, v.imag])


def _dense_bfgs_direction(g, S, Y, gamma):
    """-H g with H from the textbook BFGS inverse update (Nocedal & Wright
    eq. 6.17 / 7.19) H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T,
    rho = 1 / (y^T s), applied to the stored pairs oldest first from H0 = gamma I,
    as dense 2N x 2N matrices over the real embedding."""
    n = 2 * g.shape[0]
    H = gamma * np.eye(n)
    for s_, y_ in zip(S, Y):
        s, y = _real(s_), _real(y_)
        rho = 1.0 / (y @ s)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    d = -H @ _real(g)
    return d[: n // 2] + 1j * d[n // 2:]


def _pairs(N, m, seed):
    g = np.random.default_rng(seed)
    # y = B s with B symmetric positive definite on R^{2N}, spectrum in [2, 9]: s^T y > 0 and the newest
    # pair's s^T y / y^T y is well away from 1
    Q, _ = np.linalg.qr(g.standard_normal((2 * N, 2 * N)))
    B = Q @ np.diag(np.linspace(2.0, 9.0, 2 * N)) @ Q.T
    S, Y = [], []
    for _ in range(m):
        s = g.standard_normal(2 * N)
        y = B @ s
        S.append(s[:N] + 1j * s[N:])
        Y.append(y[:N] + 1j * y[N:])
    gr = g.standard_normal(N) + 1j * g.standard_normal(N)
    return gr, S, Y


def test_two_loop_scaling_equals_dense_bfgs():
    N = 6
    for m in (1, 2, 5):
        g, S, Y = _pairs(N, m, 10 + m)
        d = rt.two_loop(g[None], [S], [Y], None)[0]
        gamma = rt.rdot(S[-1], Y[-1]) / rt.rdot(Y[-1], Y[-1])
        assert 0.05 < gamma < 0.6  # far from 1, so the scaling matters
        ref = _dense_bfgs_direction(g, S, Y, gamma)
        assert np.max(np.abs(d - ref)) < 1e-12 * np.max(np.abs(ref))
        # planted mistakes: inverted scaling, or the oldest pair's scaling
        bad = _dense_bfgs_direction(g, S, Y, 1.0 / gamma)
        assert np.max(np.abs(d - bad)) > 1e-3 * np.max(np.abs(ref))
        if m > 1:
            g_old = rt.rdot(S[0], Y[0]) / rt.rdot(Y[0], Y[0])
            bad = _dense_bfgs_direction(g, S, Y, g_old)
            assert np.max(np.abs(d - bad)) > 1e-6 * np.max(np.abs(ref))
    # with a fixed gamma the recursion is the same dense update from gamma I
    g, S, Y = _pairs(N, 3, 99)
    d = rt.two_loop(g[None], [S], [Y], 0.7)[0]
    assert np.max(np.abs(d - _dense_bfgs_direction(g, S, Y, 0.7))) < 1e-12 * np.max(np.abs(d))
    # no pairs: -h0 g
    assert np.allclose(rt.two_loop(g[None], [[]], [[]], None, h0=0.25)[0], -0.25 * g)


def test_spectral_weights_hand_example():
    ex = json.load(open(GOLD))["spectral_weights"]
    I = np.asarray(ex["I"], dtype=np.float64)
    w = rt.spectral_weights(I, ex["tau"])
    assert np.array_equal(w, np.asarray(ex["w"], dtype=np.float64))
    # planted mistake: one mean over every row
    bad = np.minimum(I / np.mean(I), ex["tau"])
    assert not np.allclose(bad, ex["w"])


def test_acceptance_residual_hand_example():
    ex = json.load(open(GOLD))["acceptance_residual"]
    masks = _c(ex["masks"])
    t = _c(ex["t"])
    I = np.asarray(ex["I"], dtype=np.float64)
    op = ops.FFTOp(masks, ex["n1"], ex["n2"])
    rho = rt.acceptance_residual(op, I, t)
    assert np.allclose(rho, ex["rho"], rtol=0, atol=1e-15)
    # planted mistake: normalising by ||I|| instead of ||I||^2
    f = rt.intensity_loss(I, op.forward(t))
    bad = f / np.sqrt(np.sum(I.reshape(I.shape[0], -1) ** 2, axis=1))
    assert not np.allclose(bad, ex["rho"])
    # and the dense operator gives the same value
    assert np.allclose(rt.acceptance_residual(ops.DenseOp(masks, ex["n1"], ex["n2"]), I, t), ex["rho"], atol=1e-15)
