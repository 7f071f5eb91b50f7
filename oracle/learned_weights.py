"""Learned weighting of the spectral start, FP64 (test infrastructure only).

Not part of the paper (its start is Eq. backpropagation). The plain start
of this build is the truncated spectral start: the top eigenvector of
M = A^H diag(w) A with w = min(I / mean(I_p), tau). The learned form keeps
that start and replaces the truncation by a function T of the normalised
intensity x = I / mean(I_p), w = T(x), which a small network proposes and
which is trained on (intensity, row) pairs of the forward model. The
spectral method's quality depends on this preprocessing function (Mondelli
& Montanari 2017; Luo, Alghamdi & Lu 2019 give the optimum for Gaussian
designs); here it is learned for the Fourier-structured design A of
Sec. 2.2 (Eq. probingmatrix) at the data's noise level.

Pieces:
  * the table: T sampled at NT points x_b = b xmax / (NT - 1); w(x) is the
    linear interpolation between the two nearest points, x clamped to
    [0, xmax];
  * the training loss: k steps of the normalised power iteration
    u <- M u / ||M u|| from a seed v0, and minus the mean fidelity
    |t^H u_k|^2 / (||t||^2 ||u_k||^2) to the true rows; its gradient with
    respect to the table by reverse-mode differentiation through the k
    steps (written out below);
  * the network that proposes the table: per table point the features
    table_features(x) -> Linear -> GELU -> Linear -> GELU -> Linear -> T(x)
    (the layers of oracle.mlp).
"""
from __future__ import annotations

import numpy as np

from . import retrieval as rt

XMAX = 16.0  # the table covers x = I / mean(I_p) in [0, XMAX]; larger x reads the last point


def normalised(I: np.ndarray) -> np.ndarray:
    """x = I / mean(I_p) per row (a row with mean 0 divides by 1), [P, K, N]."""
    m = np.mean(I.reshape(I.shape[0], -1), axis=1)
    m = np.where(m > 0, m, 1.0)
    return I / m.reshape((-1,) + (1,) * (I.ndim - 1))


def interp_index(x: np.ndarray, nt: int, xmax: float = XMAX):
    """Lower table index i0 and fraction f in [0, 1] of every x:
    w = (1 - f) T[i0] + f T[i0 + 1] on the uniform grid of nt points."""
    s = np.clip(x, 0.0, xmax) * ((nt - 1) / xmax)
    i0 = np.minimum(np.floor(s).astype(np.int64), nt - 2)
    return i0, s - i0


def table_weights(table: np.ndarray, x: np.ndarray, xmax: float = XMAX) -> np.ndarray:
    i0, f = interp_index(x, len(table), xmax)
    return (1.0 - f) * table[i0] + f * table[i0 + 1]


def table_grid(nt: int, xmax: float = XMAX) -> np.ndarray:
    return np.arange(nt) * (xmax / (nt - 1))


def scatter_to_table(gw: np.ndarray, x: np.ndarray, nt: int, xmax: float = XMAX) -> np.ndarray:
    """Adjoint of table_weights: d/dT_b of sum_i gw_i w_i."""
    i0, f = interp_index(x, nt, xmax)
    out = np.zeros(nt)
    np.add.at(out, i0.ravel(), ((1.0 - f) * gw).ravel())
    np.add.at(out, i0.ravel() + 1, (f * gw).ravel())
    return out


def power_loss(op, I, t, v0, table, k, xmax: float = XMAX, grad: bool = True):
    """Loss = - mean_p |t_p^H u_k|^2 / (||t_p||^2 ||u_k||^2) after k normalised
    power steps u <- M u / ||M u||, M = A^H diag(T(x)) A, u_0 = v0 / ||v0||.
    Returns (loss, d loss / d table) (the gradient is None with grad=False).

    Reverse mode, with packed gradients (d/dRe + j d/dIm, Eq. derivative's
    convention) and <a, b> = Re(a^H b):
      G_{u_k} = -(2 c t / (||t||^2 ||u||^2) - 2 |c|^2 u / (||t||^2 ||u||^4)) / B,  c = t^H u_k;
      through u = y / ||y||:   G_y = (G_u - <u, G_u> u) / ||y||;
      through y = M u:         G_u(previous) = M G_y,
                               d loss / d w_i += Re(conj((A G_y)_i) (A u)_i)."""
    x = normalised(I)
    w = table_weights(table, x, xmax)
    B = I.shape[0]
    u = v0 / np.linalg.norm(v0, axis=1, keepdims=True)
    us, ns = [u], []
    for _ in range(k):
        y = op.adjoint(w * op.forward(u))
        n = np.linalg.norm(y, axis=1, keepdims=True)
        ns.append(n)
        u = y / n
        us.append(u)
    tt = np.sum(np.abs(t) ** 2, axis=1, keepdims=True)
    uu = np.sum(np.abs(u) ** 2, axis=1, keepdims=True)
    c = np.sum(np.conj(t) * u, axis=1, keepdims=True)
    fid = (np.abs(c) ** 2 / (tt * uu))[:, 0]
    loss = -float(np.mean(fid))
    if not grad:
        return loss, None
    G = -(2.0 * c * t / (tt * uu) - 2.0 * np.abs(c) ** 2 * u / (tt * uu ** 2)) / B
    gw = np.zeros_like(w)
    for j in range(k - 1, -1, -1):
        uj1 = us[j + 1]
        Gy = (G - rt.rdot(uj1, G)[:, None] * uj1) / ns[j]
        AG = op.forward(Gy)
        gw += np.real(np.conj(AG) * op.forward(us[j]))
        G = op.adjoint(w * AG)
    return loss, scatter_to_table(gw, x, len(table), xmax)


N_FEAT = 64


def table_features(xg: np.ndarray, xmax: float = XMAX) -> np.ndarray:
    """[NT] table abscissae -> [NT, 64] network inputs: smooth functions of x
    on [0, xmax] (powers, saturating and decaying forms, 48 sinusoids)."""
    u = xg / xmax
    cols = [u, np.sqrt(u), u * u, np.log1p(xg) / np.log1p(xmax), np.exp(-xg), np.exp(-xg / 4.0),
            1.0 / (1.0 + xg), xg / (1.0 + xg), np.tanh(xg - 1.0), np.tanh((xg - 3.0) / 2.0),
            np.minimum(xg, 1.0), np.minimum(xg, 2.0) / 2.0, np.minimum(xg, 3.0) / 3.0, np.minimum(xg, 5.0) / 5.0,
            np.ones_like(xg), np.exp(-xg * xg)]
    for f in range(1, 25):
        cols.append(np.sin(np.pi * f * u))
        cols.append(np.cos(np.pi * f * u))
    return np.stack(cols, axis=1)


def table_pairs(values: np.ndarray) -> np.ndarray:
    """[nt] table values -> [nt, 2] (T_b, T_{b+1} - T_b), last slope 0 (the
    layout the library reads)."""
    v = np.asarray(values, dtype=np.float64)
    return np.stack([v, np.append(np.diff(v), 0.0)], axis=1)


def network_table(params: dict, nt: int, xmax: float = XMAX, bf16=None) -> np.ndarray:
    """The network's table values T(x_b) at the nt grid points: features ->
    Linear -> GELU -> Linear -> GELU -> Linear (oracle.mlp.forward). `bf16`,
    if given, is a rounding function applied where the device stores BF16
    (features, weights, hidden activations), so that only the accumulation
    order differs."""
    from . import mlp
    X = table_features(table_grid(nt, xmax), xmax)
    if bf16 is None:
        o, _ = mlp.forward(params, X)
        return o[:, 0]
    p = params
    h1 = bf16(mlp.gelu(bf16(X) @ bf16(p["W1"]) + p["b1"]))
    h2 = bf16(mlp.gelu(h1 @ bf16(p["W2"]) + p["b2"]))
    return (h2 @ bf16(p["W3"]) + p["b3"])[:, 0]
