"""Per-row TM retrieval, FP64 (test infrastructure only).

Follows Sec. 2.2 of the paper: the per-pixel least-squares problem
f(t) = || I - |A t|^2 ||^2 (Eq. optTMsmall2), its gradient
(Eq. derivative, App. A), the back-propagation start (Eq.
backpropagation) and Algorithm 1 (f, gradient, L-BFGS direction, update,
stop at maxiter). Also the amplitude-projection form (error reduction, the
Gerchberg-Saxton / Fienup family the paper's Discussion names), its cyclic
form (one mask's projection at a time) and a spectral start.

Readings where the paper is silent:
  * Gradient packing: the paper's (df/dt)^H = df/dx + j df/dy, i.e. the real
    gradient over R^{2N} stored as a complex vector; inner products over
    R^{2N} are Re(a^H b).
  * L-BFGS (Nocedal & Wright Alg. 7.4, Liu & Nocedal 1989, both cited by
    the paper): memory m (default 5), H0 = gamma I with
    gamma = s^T y / y^T y of the newest pair (or a fixed gamma on request),
    pairs with s^T y <= 0 are skipped, a non-descent direction resets the
    history and falls back to the negative gradient.
  * Line search: f(t + a d) is a quartic in a; its exact minimiser over
    a > 0 is taken among the real roots of the cubic f'(a) = 0 (smallest
    f, ties to the smaller a).
  * Zero field in the projection: y/|y| := 1 where y = 0.
  * Spectral start (plain starts are random or spectral; the paper's
    back-propagation start does not reach the truth at K = 4): power
    iteration on A^H diag(w) A with truncated weights
    w = min(I / mean(I_p), tau), optionally heavy-ball accelerated, then
    scaled so that ||t||^2 = sum(I_p) / (K N) (Parseval, A^H A = K N I);
    or the same eigenvector estimated by Lanczos steps (the Ritz vector of
    the largest Ritz value, no reorthogonalisation).
  * Fidelity |t_hat^H t|^2 / (||t_hat||^2 ||t||^2), invariant to a row's
    phase (Sec. 2.3, Eq. phaseoffset) and scale.
"""
from __future__ import annotations

import numpy as np


def rdot(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Inner product over R^{2N} of complex-packed vectors, per row: Re(a^H b)."""
    return np.real(np.sum(np.conj(a) * b, axis=-1))


def intensity_loss(I: np.ndarray, y: np.ndarray) -> np.ndarray:
    """f = sum (I - |y|^2)^2 per row (Eq. optTMsmall2)."""
    r = I - np.abs(y) ** 2
    return np.sum(r.reshape(r.shape[0], -1) ** 2, axis=1)


def amplitude_residual(I: np.ndarray, y: np.ndarray) -> np.ndarray:
    """sum (sqrt(I) - |y|)^2 per row: the amplitude-based cost the paper's
    Discussion names for Poisson noise."""
    d = np.sqrt(I) - np.abs(y)
    return np.sum(d.reshape(d.shape[0], -1) ** 2, axis=1)


def intensity_grad(op, I: np.ndarray, t: np.ndarray):
    """(df/dt)^H = -4 A^H diag(A t) (I - |A t|^2) (Eq. derivative).
    Returns (f, grad, y)."""
    y = op.forward(t)
    r = I - np.abs(y) ** 2
    g = -4.0 * op.adjoint(y * r)
    return np.sum(r.reshape(r.shape[0], -1) ** 2, axis=1), g, y


def amplitude_grad(op, I: np.ndarray, t: np.ndarray):
    """Amplitude cost f_a = sum (sqrt(I) - |A t|)^2 (the Poisson-noise cost of
    the Discussion) and its packed gradient -2 A^H((sqrt(I) - |y|) y/|y|),
    with y/|y| := 1 at y = 0. Returns (f_a, grad, y)."""
    y = op.forward(t)
    r = np.sqrt(I) - np.abs(y)
    g = -2.0 * op.adjoint(r * phase_of(y))
    return np.sum(r.reshape(r.shape[0], -1) ** 2, axis=1), g, y


AMP_STEPS = 2.0 ** np.arange(-3, 5)  # trial steps of the amplitude line search: 1/8 .. 16


def amplitude_step(I: np.ndarray, y: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Line search of the amplitude L-BFGS along d with y = A t, z = A d:
    f_a(t + a d) = sum (sqrt(I) - |y + a z|)^2 at the trial steps AMP_STEPS;
    the smallest value wins (ties to the smaller step) if it is below
    f_a(t), else the step is 0. Returns a per row."""
    amp = np.sqrt(I)
    ax = tuple(range(1, I.ndim))
    f0 = np.sum((amp - np.abs(y)) ** 2, axis=ax)
    fs = np.stack([np.sum((amp - np.abs(y + a * z)) ** 2, axis=ax) for a in AMP_STEPS], axis=1)
    j = np.argmin(fs, axis=1)  # first minimum = smaller step on ties
    best = fs[np.arange(fs.shape[0]), j]
    return np.where(best < f0, AMP_STEPS[j], 0.0)


def acceptance_residual(op, I: np.ndarray, t: np.ndarray) -> np.ndarray:
    """rho_p = ||I_p - |A t_p|^2||^2 / ||I_p||^2, a ground-truth-free
    per-row error flag."""
    f = intensity_loss(I, op.forward(t))
    return f / np.sum(I.reshape(I.shape[0], -1) ** 2, axis=1)


def phase_of(y: np.ndarray) -> np.ndarray:
    """y / |y| with the zero-field convention 1 at y == 0."""
    a = np.abs(y)
    out = np.ones_like(y)
    nz = a > 0
    out[nz] = y[nz] / a[nz]
    return out


def er_step(op, I: np.ndarray, t: np.ndarray) -> np.ndarray:
    """One projection (error-reduction) step: keep the measured amplitudes,
    keep the current phases, project back: t <- A^H(sqrt(I) y/|y|) / (K N).
    A A^H / (K N) is the orthogonal projector onto range(A), so the amplitude
    residual cannot increase."""
    y = op.forward(t)
    return op.adjoint(np.sqrt(I) * phase_of(y)) / (op.K * op.N)


def er_accelerated(op, I: np.ndarray, t0: np.ndarray, iters: int, beta: float) -> np.ndarray:
    """Error reduction with Nesterov momentum: z = t + beta (t - t_prev),
    t_new = er_step(z); t_prev starts equal to t0 (so the first step is plain
    ER). ER is a gradient step of length 1/(K N) on the amplitude cost, and
    this is Nesterov's acceleration of that step. beta = 0 gives plain ER."""
    t = np.array(t0, dtype=np.complex128)
    tp = t.copy()
    for _ in range(iters):
        z = t + beta * (t - tp)
        tp, t = t, er_step(op, I, z)
    return t


def er_cyclic(masks: np.ndarray, n1: int, n2: int, I: np.ndarray, t0: np.ndarray, iters: int) -> np.ndarray:
    """Error reduction with the masks taken one at a time (cyclic projections;
    a solver chosen here, not the paper's): a sweep projects the row onto the
    measurement set of each mask in turn,
        y = F(psi_m t),  t <- conj(psi_m) F^H(sqrt(I_m) y/|y|) / N,  m = 1..K,
    with F the unnormalised 2-D DFT (F^H F = N). F diag(psi_m) / sqrt(N) is
    unitary, so each update is the nearest point of
    {t : |F(psi_m t)|^2 = I_m} (the plain ER step averages the K such
    projections instead). y/|y| := 1 where y = 0."""
    masks = np.asarray(masks, dtype=np.complex128)
    K, N = masks.shape
    t = np.array(np.atleast_2d(t0), dtype=np.complex128)
    P = t.shape[0]
    amp = np.sqrt(np.maximum(np.asarray(I, dtype=np.float64).reshape(P, K, N), 0.0))
    for _ in range(iters):
        for m in range(K):
            y = np.fft.fft2((masks[m][None, :] * t).reshape(P, n1, n2)).reshape(P, N)
            w = amp[:, m, :] * phase_of(y)
            t = np.conj(masks[m])[None, :] * np.fft.ifft2(w.reshape(P, n1, n2)).reshape(P, N)
    return t


def er_cyclic_sweep_sums(masks: np.ndarray, n1: int, n2: int, I: np.ndarray, t0: np.ndarray):
    """The residual sums of one sweep from t0, each mask's term taken at the
    iterate its projection starts from: (sum_m ||sqrt(I_m) - |y_m|||^2,
    sum_m ||I_m - |y_m|^2||^2) per row."""
    masks = np.asarray(masks, dtype=np.complex128)
    K, N = masks.shape
    t = np.array(np.atleast_2d(t0), dtype=np.complex128)
    P = t.shape[0]
    Iv = np.asarray(I, dtype=np.float64).reshape(P, K, N)
    amp = np.sqrt(np.maximum(Iv, 0.0))
    sa = np.zeros(P)
    si = np.zeros(P)
    for m in range(K):
        y = np.fft.fft2((masks[m][None, :] * t).reshape(P, n1, n2)).reshape(P, N)
        sa += np.sum((amp[:, m, :] - np.abs(y)) ** 2, axis=1)
        si += np.sum((Iv[:, m, :] - np.abs(y) ** 2) ** 2, axis=1)
        t = np.conj(masks[m])[None, :] * np.fft.ifft2((amp[:, m, :] * phase_of(y)).reshape(P, n1, n2)).reshape(P, N)
    return sa, si


def backprop_start(op, I: np.ndarray) -> np.ndarray:
    """t0 = (A^H A)^{-1} A^H sqrt(I) = A^H sqrt(I) / (K N) (Eq. backpropagation)."""
    return op.adjoint(np.sqrt(I)) / (op.K * op.N)


def spectral_weights(I: np.ndarray, tau: float) -> np.ndarray:
    m = np.mean(I.reshape(I.shape[0], -1), axis=1)
    m = np.where(m > 0, m, 1.0)
    return np.minimum(I / m[:, None, None], tau)


def spectral_start(op, I: np.ndarray, v0: np.ndarray, iters: int, tau: float = 3.0,
                   momentum: float = 0.0, lower: float | None = None) -> np.ndarray:
    """Truncated spectral start: power iteration on M = A^H diag(w) A from v0
    (unit-normalised each step), then scaled to ||t||^2 = sum(I)/(K N).

    momentum = c > 0 selects the heavy-ball power method (Xu et al.,
    "Accelerated stochastic power iteration", 2018): x_{k+1} = M x_k -
    beta_k x_{k-1} with beta_k = (c lambda_k)^2 / 4 and lambda_k the
    Rayleigh quotient of the current unit vector; both x_{k+1} and x_k are
    divided by ||x_{k+1}|| so the recurrence keeps its ratios. It converges
    to the same top eigenvector in fewer steps. c = 0 is plain power
    iteration.

    The recurrence is the Chebyshev-type iteration for the rest of the
    spectrum assumed in [-c lambda, c lambda]. M is positive semidefinite,
    so the rest lies in [0, c lambda]: lower = l centres the iteration on
    the interval [l lambda, c lambda], x_{k+1} = (M - sigma_k) x_k -
    beta_k x_{k-1} with sigma_k = (c + l) lambda_k / 2 and beta_k =
    ((c - l) lambda_k / 2)^2 / 4 (the shifted matrix has the same
    eigenvectors). lower = None is l = -c (no shift)."""
    w = spectral_weights(I, tau)
    v = np.array(v0, dtype=np.complex128)
    n = np.linalg.norm(v, axis=1)
    v = v / np.where(n > 0, n, 1.0)[:, None]
    vp = np.zeros_like(v)
    for _ in range(iters):
        Mv = op.adjoint(w * op.forward(v))
        lam = rdot(v, Mv)
        lo = -momentum if lower is None else lower
        sigma = (momentum + lo) * lam / 2.0
        beta = ((momentum - lo) * lam / 2.0) ** 2 / 4.0
        x = Mv - sigma[:, None] * v - beta[:, None] * vp
        n = np.linalg.norm(x, axis=1)
        n = np.where(n > 0, n, 1.0)[:, None]
        vp = v / n
        v = x / n
    scale = np.sqrt(np.sum(I.reshape(I.shape[0], -1), axis=1) / (op.K * op.N))
    return v * scale[:, None]


def spectral_lanczos(op, I: np.ndarray, v0: np.ndarray, iters: int, tau: float = 3.0, basis: bool = False,
                     weights: np.ndarray | None = None):
    """Truncated spectral start by the Lanczos method (a choice made here):
    `iters` Lanczos steps on M = A^H diag(w) A (w as in spectral_start) from
    v_1 = v0 / ||v0||,
        x = M v_j - alpha_j v_j - beta_j v_{j-1},  alpha_j = Re(v_j^H M v_j),
        beta_{j+1} = ||x||,  v_{j+1} = x / beta_{j+1}   (beta_1 = 0),
    then the eigenvector y of the largest eigenvalue of the real symmetric
    tridiagonal T (diagonal alpha_1..alpha_k, off-diagonal beta_2..beta_k),
    sign fixed by y_1 >= 0, and t = sum_j y_j v_j, normalised and scaled to
    ||t||^2 = sum(I_p) / (K N). No reorthogonalisation. With basis=True also
    returns (alpha [P][k], beta [P][k] (beta[:, j] = beta_{j+1}), V [k+1][P][N]).
    `weights` [P, K, N] replaces the truncated weights (the learned form)."""
    w = spectral_weights(I, tau) if weights is None else weights
    v = np.array(v0, dtype=np.complex128)
    P = v.shape[0]
    n = np.linalg.norm(v, axis=1)
    v = v / np.where(n > 0, n, 1.0)[:, None]
    vp = np.zeros_like(v)
    bp = np.zeros(P)
    V = [v]
    al = np.zeros((P, iters))
    be = np.zeros((P, iters))
    for j in range(iters):
        Mv = op.adjoint(w * op.forward(v))
        a = rdot(v, Mv)
        x = Mv - a[:, None] * v - bp[:, None] * vp
        b = np.linalg.norm(x, axis=1)
        al[:, j] = a
        be[:, j] = b
        vp, bp = v, b
        v = x / np.where(b > 0, b, 1.0)[:, None]
        V.append(v)
    t = np.zeros_like(v)
    for p in range(P):
        Tm = np.diag(al[p]) + np.diag(be[p, :-1], 1) + np.diag(be[p, :-1], -1)
        ev, vec = np.linalg.eigh(Tm)
        y = vec[:, -1] * (1.0 if vec[0, -1] >= 0 else -1.0)
        t[p] = sum(y[j] * V[j][p] for j in range(iters))
    nt = np.linalg.norm(t, axis=1)
    scale = np.sqrt(np.sum(I.reshape(P, -1), axis=1) / (op.K * op.N))
    t = t / np.where(nt > 0, nt, 1.0)[:, None] * scale[:, None]
    if basis:
        return t, al, be, np.array(V)
    return t


def fidelity(t_hat: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Per-row |t_hat^H t|^2 / (||t_hat||^2 ||t||^2)."""
    num = np.abs(np.sum(np.conj(t_hat) * t, axis=-1)) ** 2
    den = np.sum(np.abs(t_hat) ** 2, axis=-1) * np.sum(np.abs(t) ** 2, axis=-1)
    return num / np.where(den > 0, den, 1.0)


def quartic_coeffs(I: np.ndarray, y: np.ndarray, z: np.ndarray):
    """Coefficients of phi(a) = f(t + a d) - f(t) = c1 a + c2 a^2 + c3 a^3 + c4 a^4,
    with y = A t, z = A d, r = I - |y|^2, b = Re(conj(y) z), c = |z|^2:
    |y + a z|^2 = |y|^2 + 2ab + a^2 c, so f(a) = sum (r - 2ab - a^2 c)^2."""
    r = I - np.abs(y) ** 2
    b = np.real(np.conj(y) * z)
    c = np.abs(z) ** 2
    ax = tuple(range(1, r.ndim))
    c1 = -4.0 * np.sum(r * b, axis=ax)
    c2 = np.sum(4.0 * b * b - 2.0 * r * c, axis=ax)
    c3 = 4.0 * np.sum(b * c, axis=ax)
    c4 = np.sum(c * c, axis=ax)
    return c1, c2, c3, c4


def exact_step(c1: float, c2: float, c3: float, c4: float) -> float:
    """Minimiser over a > 0 of c1 a + c2 a^2 + c3 a^3 + c4 a^4: among the
    real positive roots of 4 c4 a^3 + 3 c3 a^2 + 2 c2 a + c1 = 0 take the
    one of smallest value (ties: smaller a). Returns 0 when there is none."""
    if not (c4 > 0):
        if c2 > 0 and c1 < 0:
            return -c1 / (2 * c2)
        return 0.0
    roots = np.roots([4 * c4, 3 * c3, 2 * c2, c1])
    cand = []
    for rt in roots:
        if abs(rt.imag) <= 1e-7 * max(1.0, abs(rt)) and rt.real > 0:
            a = rt.real
            cand.append((c1 * a + c2 * a * a + c3 * a ** 3 + c4 * a ** 4, a))
    if not cand:
        return 0.0
    cand.sort()
    return float(cand[0][1])


def lbfgs_core(eval_fg, line_min, t0: np.ndarray, iters: int, m: int = 5,
               gamma: float | None = None, callback=None, h0: float = 1.0,
               reset_on_zero: bool = False, events: dict | None = None):
    """Generic per-row L-BFGS loop of Algorithm 1: `eval_fg(t) -> (f, g, aux)`
    gives the error and packed gradient, `line_min(t, d, aux) -> alpha` the
    step along d. With an empty history the direction is -h0 g (also after a
    non-descent reset); reset_on_zero drops a row's history when its step is
    0. Returns (t, per-iteration f history [iters+1, P]). If `events` is a
    dict it receives per-row counts of what happened to the history:
    "skipped" (nonzero steps whose pair had s^T y <= 0), "evicted" (pairs
    dropped because m were stored), "zero_steps" and "resets" (non-descent)."""
    t = np.array(t0, dtype=np.complex128)
    P = t.shape[0]
    S = [[] for _ in range(P)]
    Y = [[] for _ in range(P)]
    f, g, aux = eval_fg(t)
    hist = [f.copy()]
    ev = {k: np.zeros(P, dtype=np.int64) for k in ("skipped", "evicted", "zero_steps", "resets")}
    for _ in range(iters):
        d = two_loop(g, S, Y, gamma, h0)
        slope = rdot(g, d)
        bad = ~(slope < 0)
        if np.any(bad):
            for p in np.nonzero(bad)[0]:
                S[p], Y[p] = [], []
            d[bad] = -h0 * g[bad]
            ev["resets"] += bad
        alpha = line_min(t, d, aux)
        ev["zero_steps"] += alpha == 0
        if reset_on_zero:
            for p in np.nonzero(alpha == 0)[0]:
                S[p], Y[p] = [], []
        t_new = t + alpha[:, None] * d
        f_new, g_new, aux_new = eval_fg(t_new)
        s_vec = t_new - t
        y_vec = g_new - g
        sy = rdot(s_vec, y_vec)
        for p in range(P):
            if sy[p] > 0:
                S[p].append(s_vec[p])
                Y[p].append(y_vec[p])
                if len(S[p]) > m:
                    S[p].pop(0)
                    Y[p].pop(0)
                    ev["evicted"][p] += 1
            elif alpha[p] != 0:
                ev["skipped"][p] += 1
        t, f, g, aux = t_new, f_new, g_new, aux_new
        hist.append(f.copy())
        if callback is not None:
            callback(t)
    if events is not None:
        events.update(ev)
    return t, np.array(hist)


def lbfgs(op, I: np.ndarray, t0: np.ndarray, iters: int, m: int = 5,
          gamma: float | None = None, callback=None, events: dict | None = None):
    """Algorithm 1 of the paper for every row at once: per iteration the
    error and gradient at the current t (Eq. optTMsmall2, Eq. derivative),
    an L-BFGS direction from the last m (s, y) pairs (two-loop recursion
    over R^{2N}), the exact line search on the quartic, and the update
    t <- t + a d (the paper's t - Delta t). Stops at `iters` (maxiter).
    Returns (t, per-iteration f history [iters+1, P])."""

    def eval_fg(t):
        return intensity_grad(op, I, t)

    def line_min(t, d, y):
        z = op.forward(d)
        c1, c2, c3, c4 = quartic_coeffs(I, y, z)
        return np.array([exact_step(c1[p], c2[p], c3[p], c4[p]) for p in range(t.shape[0])])

    return lbfgs_core(eval_fg, line_min, t0, iters, m, gamma, callback, events=events)


def two_loop(g: np.ndarray, S, Y, gamma: float | None, h0: float = 1.0) -> np.ndarray:
    """L-BFGS two-loop recursion per row (Nocedal & Wright Alg. 7.4):
    returns d = -H g with the inverse-Hessian approximation built from the
    stored pairs, oldest first in S[p], Y[p]; H = h0 I with no pairs."""
    d = np.empty_like(g)
    for p in range(g.shape[0]):
        q = g[p].copy()
        a = []
        for s_, y_ in zip(reversed(S[p]), reversed(Y[p])):
            rho = 1.0 / np.real(np.vdot(y_, s_))
            ai = rho * np.real(np.vdot(s_, q))
            q = q - ai * y_
            a.append(ai)
        if gamma is not None:
            q = q * gamma
        elif S[p]:
            q = q * (np.real(np.vdot(S[p][-1], Y[p][-1])) / np.real(np.vdot(Y[p][-1], Y[p][-1])))
        else:
            q = q * h0
        for (s_, y_), ai in zip(zip(S[p], Y[p]), reversed(a)):
            rho = 1.0 / np.real(np.vdot(y_, s_))
            b = rho * np.real(np.vdot(y_, q))
            q = q + (ai - b) * s_
        d[p] = -q
    return d


def lbfgs_amplitude(op, I: np.ndarray, t0: np.ndarray, iters: int, m: int = 5, callback=None,
                    events: dict | None = None):
    """L-BFGS on the amplitude cost (the Poisson-noise variant the Discussion
    names, same two-loop recursion as Algorithm 1): gradient amplitude_grad,
    line search amplitude_step over the trial steps, and with no stored pairs
    the direction -g/(2KN), along which the unit step is one error-reduction
    step (the amplitude gradient is 2KN (t - ER(t))). A row whose line search
    finds no decrease drops its history, so its next step is again of that
    kind, which never increases f_a. Returns (t, f_a history)."""

    def eval_fg(t):
        return amplitude_grad(op, I, t)

    def line_min(t, d, y):
        return amplitude_step(I, y, op.forward(d))

    return lbfgs_core(eval_fg, line_min, t0, iters, m, None, callback, h0=1.0 / (2.0 * op.K * op.N),
                      reset_on_zero=True, events=events)
