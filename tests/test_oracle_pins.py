"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics (library special cases, closed forms, invariants, brute force,
hand-worked examples). CPU only."""
import json
import os

import numpy as np
import pytest

import tm_synth
from oracle import operators as ops
from oracle import retrieval as rt

GOLD = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def cplx(a):
    a = np.asarray(a, dtype=np.float64)
    return a[..., 0] + 1j * a[..., 1]


def small_problem(n1=4, n2=4, K=4, P=3, seed=11):
    g = np.random.default_rng(seed)
    N = n1 * n2
    masks = np.exp(2j * np.pi * g.random((K, N)))
    t = (g.standard_normal((P, N)) + 1j * g.standard_normal((P, N))) / np.sqrt(2)
    return masks, t, g


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 16, 12])
def test_dft_matrix_is_numpy_fft(n):
    # the unnormalised forward DFT is numpy's fft (library special case)
    F = ops.dft_matrix(n)
    assert np.max(np.abs(F - np.fft.fft(np.eye(n), axis=0))) < 1e-12


def test_dft2_is_fft2_on_row_major_grid():
    g = np.random.default_rng(0)
    x = g.standard_normal((4, 8)) + 1j * g.standard_normal((4, 8))
    F = ops.dft2_matrix(4, 8)
    assert np.max(np.abs(F @ x.ravel() - np.fft.fft2(x).ravel())) < 1e-12


@pytest.mark.parametrize("n1,n2", [(8, 8), (4, 8), (1, 16), (16, 1), (2, 32)])
def test_fft_operator_equals_dense(n1, n2):
    masks, t, _ = small_problem(n1, n2, K=4, P=3)
    d = ops.DenseOp(masks, n1, n2)
    f = ops.FFTOp(masks, n1, n2)
    y1, y2 = d.forward(t), f.forward(t)
    assert np.max(np.abs(y1 - y2)) <= 1e-12 * np.max(np.abs(y1))
    w = np.random.default_rng(3).standard_normal(y1.shape) + 0j
    x1, x2 = d.adjoint(w), f.adjoint(w)
    assert np.max(np.abs(x1 - x2)) <= 1e-12 * np.max(np.abs(x1))


def test_adjoint_identity_and_gram():
    masks, t, g = small_problem(4, 4, K=3, P=2)
    d = ops.DenseOp(masks, 4, 4)
    y = g.standard_normal((2, 3, 16)) + 1j * g.standard_normal((2, 3, 16))
    lhs = np.sum(np.conj(d.forward(t)) * y, axis=(1, 2))
    rhs = np.sum(np.conj(t) * d.adjoint(y), axis=1)
    assert np.max(np.abs(lhs - rhs)) < 1e-10
    G = d.A.conj().T @ d.A
    assert np.max(np.abs(G - 3 * 16 * np.eye(16))) < 1e-10


def test_hand_forward_examples():
    gold = json.load(open(GOLD))
    for ex in gold["forward"]:
        masks = cplx(ex["masks"])
        t = cplx(ex["t"])[None, :]
        for Op in (ops.DenseOp, ops.FFTOp):
            I = ops.intensities(Op(masks, ex["n1"], ex["n2"]), t).ravel()
            assert np.allclose(I, ex["I"], atol=1e-12), ex["name"]


def test_hand_gradient_example():
    gold = json.load(open(GOLD))
    for ex in gold["gradient"]:
        op = ops.DenseOp(cplx(ex["masks"]), ex["n1"], ex["n2"])
        I = np.asarray(ex["I"], dtype=float).reshape(1, op.K, op.N)
        f, g, _ = rt.intensity_grad(op, I, cplx(ex["t"]))
        assert abs(f[0] - ex["f"]) < 1e-12
        assert np.allclose(g, cplx(ex["grad"]), atol=1e-12)


def test_intensity_phase_invariance():
    # multiplying a row by e^{j phi0} leaves every intensity unchanged (Sec. 2.3)
    masks, t, _ = small_problem(4, 8, K=4, P=2)
    op = ops.FFTOp(masks, 4, 8)
    I = ops.intensities(op, t)
    t2 = t * np.exp(1j * np.array([0.7, -2.1]))[:, None]
    assert np.max(np.abs(ops.intensities(op, t2) - I)) < 1e-10 * I.max()
    assert np.all(rt.intensity_loss(I, op.forward(t2)) < 1e-16 * np.sum(I ** 2))


def test_gradient_matches_central_differences():
    # pins the factor -4, the sign and the packing d/dx + j d/dy of Eq. derivative
    masks, t, g = small_problem(2, 4, K=4, P=1, seed=5)
    op = ops.DenseOp(masks, 2, 4)
    I = ops.intensities(op, t + 0.3 * (g.standard_normal(t.shape) + 1j * g.standard_normal(t.shape)))
    x = t + 0.2 * g.standard_normal(t.shape)
    f0, grad, _ = rt.intensity_grad(op, I, x)
    h = 1e-6
    num = np.zeros(x.shape[1], dtype=complex)
    for i in range(x.shape[1]):
        for part, unit in ((0, 1.0), (1, 1j)):
            e = np.zeros_like(x)
            e[0, i] = unit * h
            fp = rt.intensity_loss(I, op.forward(x + e))[0]
            fm = rt.intensity_loss(I, op.forward(x - e))[0]
            num[i] += (fp - fm) / (2 * h) * (1 if part == 0 else 1j)
    assert np.max(np.abs(num - grad[0])) < 1e-5 * np.max(np.abs(grad))


def test_quartic_expansion_matches_direct_evaluation():
    masks, t, g = small_problem(4, 4, K=4, P=2, seed=9)
    op = ops.FFTOp(masks, 4, 4)
    I = ops.intensities(op, t)
    x = t + 0.5 * (g.standard_normal(t.shape) + 1j * g.standard_normal(t.shape))
    d = g.standard_normal(t.shape) + 1j * g.standard_normal(t.shape)
    y, z = op.forward(x), op.forward(d)
    c1, c2, c3, c4 = rt.quartic_coeffs(I, y, z)
    f0 = rt.intensity_loss(I, y)
    for a in (-0.3, 0.01, 0.2, 1.1):
        direct = rt.intensity_loss(I, op.forward(x + a * d))
        poly = f0 + c1 * a + c2 * a ** 2 + c3 * a ** 3 + c4 * a ** 4
        assert np.allclose(direct, poly, rtol=1e-10)
    # c1 is the directional derivative Re(grad^H d)
    _, grad, _ = rt.intensity_grad(op, I, x)
    assert np.allclose(c1, rt.rdot(grad, d), rtol=1e-10)


def test_exact_step_beats_dense_grid():
    g = np.random.default_rng(2)
    for _ in range(200):
        c4 = g.random() + 1e-3
        c3, c2 = g.standard_normal(2) * 3
        c1 = -abs(g.standard_normal()) - 1e-3  # descent
        a = rt.exact_step(c1, c2, c3, c4)
        grid = np.linspace(0, 20, 200001)
        phi = c1 * grid + c2 * grid ** 2 + c3 * grid ** 3 + c4 * grid ** 4
        best = phi.min()
        va = c1 * a + c2 * a ** 2 + c3 * a ** 3 + c4 * a ** 4
        assert a > 0
        assert va <= best + 1e-6 * (1 + abs(best))


def test_lbfgs_on_quadratic_reproduces_cg():
    # Nazareth (1979): with exact line search and a fixed H0 = gamma I, BFGS-type
    # updates generate the conjugate-gradient iterates on a convex quadratic.
    g = np.random.default_rng(4)
    N = 6
    B = g.standard_normal((N, N)) + 1j * g.standard_normal((N, N))
    H = B.conj().T @ B + 0.5 * np.eye(N)       # Hermitian PD: real-symmetric on R^{2N}
    b = g.standard_normal((1, N)) + 1j * g.standard_normal((1, N))
    x0 = np.zeros((1, N), dtype=complex)

    def eval_fg(t):
        gr = t @ H.T - b                         # packed gradient H t - b
        f = 0.5 * np.real(np.sum(np.conj(t) * (t @ H.T), 1)) - np.real(np.sum(np.conj(b) * t, 1))
        return f, gr, None

    def line_min(t, d, aux):
        gr = t @ H.T - b
        return -rt.rdot(gr, d) / rt.rdot(d, d @ H.T)

    xs = []
    rt.lbfgs_core(eval_fg, line_min, x0, 5, m=10, gamma=1.0, callback=lambda t: xs.append(t.copy()))
    # textbook linear CG over R^{2N} with <a, b> = Re(a^H b)
    x = x0.copy()
    r = b - x @ H.T
    p = r.copy()
    for k in range(5):
        Hp = p @ H.T
        a = rt.rdot(r, r) / rt.rdot(p, Hp)
        x = x + a[:, None] * p
        rn = r - a[:, None] * Hp
        beta = rt.rdot(rn, rn) / rt.rdot(r, r)
        p = rn + beta[:, None] * p
        r = rn
        assert np.max(np.abs(xs[k] - x)) < 1e-8 * max(1.0, np.max(np.abs(x)))


def test_er_amplitude_residual_never_increases():
    # A A^H / (K N) is an orthogonal projector, so error reduction cannot
    # increase the amplitude residual (Fienup 1982)
    c = 1
    g0, g1, g3 = tm_synth.rng(c, 0), tm_synth.rng(c, 1), tm_synth.rng(c, 3)
    masks = tm_synth.mask_phases(4, 64, g0)
    T = tm_synth.tm_iid(32, 64, g1)
    op = ops.FFTOp(masks, 8, 8)
    I = ops.intensities(op, T)
    t = tm_synth.random_start(32, 64, I.reshape(32, -1).sum(1) / (4 * 64 * 64), g3)
    prev = rt.amplitude_residual(I, op.forward(t))
    for _ in range(200):
        t = rt.er_step(op, I, t)
        cur = rt.amplitude_residual(I, op.forward(t))
        assert np.all(cur <= prev * (1 + 1e-12) + 1e-12)
        prev = cur


def test_backprop_start_is_pseudo_inverse():
    # (A^H A)^{-1} A^H sqrt(I) = A^H sqrt(I) / (K N) (Eq. backpropagation)
    masks, t, _ = small_problem(2, 4, K=3, P=2)
    d = ops.DenseOp(masks, 2, 4)
    I = ops.intensities(d, t)
    ref = np.linalg.lstsq(d.A, np.sqrt(I).reshape(2, -1).T, rcond=None)[0].T
    assert np.max(np.abs(rt.backprop_start(d, I) - ref)) < 1e-12


def test_spectral_start_converges_to_top_eigenvector():
    masks, t, g = small_problem(2, 4, K=4, P=1, seed=21)
    d = ops.DenseOp(masks, 2, 4)
    I = ops.intensities(d, t)
    w = rt.spectral_weights(I, 3.0).reshape(-1)
    M = d.A.conj().T @ (w[:, None] * d.A)
    ev, V = np.linalg.eigh(M)
    ratio = ev[-2] / ev[-1]
    iters = int(np.ceil(np.log(1e-10) / np.log(ratio)))
    assert iters < 5000
    v0 = g.standard_normal((1, 8)) + 1j * g.standard_normal((1, 8))
    v = rt.spectral_start(d, I, v0, iters)
    ov = np.abs(np.vdot(V[:, -1], v[0])) ** 2 / np.vdot(v[0], v[0]).real
    assert ov > 1 - 1e-8
    assert abs(np.linalg.norm(v) ** 2 - I.sum() / (4 * 8)) < 1e-9 * I.sum()


def test_fidelity_invariances():
    g = np.random.default_rng(1)
    t = g.standard_normal((3, 10)) + 1j * g.standard_normal((3, 10))
    assert np.allclose(rt.fidelity(t, t), 1.0)
    assert np.allclose(rt.fidelity(2.5 * np.exp(1j * 0.3) * t, t), 1.0)
    u = g.standard_normal((3, 10)) + 1j * g.standard_normal((3, 10))
    f = rt.fidelity(u, t)
    assert np.all((f >= 0) & (f <= 1))


def test_noiseless_recovery_lbfgs_spectral():
    # noiseless data: the exact answer is the truth up to one phase per row
    # (Sec. 2.3). Spectral start + Algorithm 1 reaches it.
    c = 1
    masks = tm_synth.mask_phases(4, 64, tm_synth.rng(c, 0))
    T = tm_synth.tm_iid(32, 64, tm_synth.rng(c, 1))
    op = ops.FFTOp(masks, 8, 8)
    I = ops.intensities(op, T)
    v0 = tm_synth.random_start(32, 64, np.ones(32), tm_synth.rng(c, 3))
    t0 = rt.spectral_start(op, I, v0, 50)
    t, hist = rt.lbfgs(op, I, t0, 200)
    F = rt.fidelity(t, T)
    ok = F >= 0.9999
    assert ok.mean() >= 0.9, F
    # f never increases under the exact line search
    assert np.all(np.diff(hist, axis=0) <= 1e-9 * hist[:-1] + 1e-20)
    # the ground-truth-free residual flags exactly the unrecovered rows
    rho = rt.acceptance_residual(op, I, t)
    assert np.all(rho[ok] < 1e-6)


def test_truth_has_zero_residual_and_gradient():
    masks, t, _ = small_problem(4, 4, K=4, P=2)
    op = ops.FFTOp(masks, 4, 4)
    I = ops.intensities(op, t)
    f, g, _ = rt.intensity_grad(op, I, t)
    assert np.all(f < 1e-20 * np.sum(I ** 2))
    assert np.max(np.abs(g)) < 1e-9 * np.max(I)
    assert np.all(rt.acceptance_residual(op, I, t) < 1e-24)


def test_more_masks_recover_more_rows():
    # qualitative trend of Sec. 3: few masks fail, more masks succeed
    frac = {}
    for K in (3, 8):
        masks = tm_synth.mask_phases(K, 64, tm_synth.rng(100 + K, 0))
        T = tm_synth.tm_iid(16, 64, tm_synth.rng(100 + K, 1))
        op = ops.FFTOp(masks, 8, 8)
        I = ops.intensities(op, T)
        t0 = rt.spectral_start(op, I, tm_synth.random_start(16, 64, np.ones(16), tm_synth.rng(100 + K, 3)), 30)
        t, _ = rt.lbfgs(op, I, t0, 100)
        frac[K] = np.mean(rt.fidelity(t, T) > 0.999)
    assert frac[8] >= 0.99 and frac[3] < frac[8]


def test_momentum_power_iteration_reaches_same_eigenvector():
    masks, t, g = small_problem(2, 4, K=4, P=1, seed=21)
    d = ops.DenseOp(masks, 2, 4)
    I = ops.intensities(d, t)
    w = rt.spectral_weights(I, 3.0).reshape(-1)
    ev, V = np.linalg.eigh(d.A.conj().T @ (w[:, None] * d.A))
    v0 = g.standard_normal((1, 8)) + 1j * g.standard_normal((1, 8))
    v = rt.spectral_start(d, I, v0, 400, momentum=0.98 * ev[-2] / ev[-1])
    assert np.abs(np.vdot(V[:, -1], v[0])) ** 2 / np.vdot(v[0], v[0]).real > 1 - 1e-8


def test_accelerated_er_special_cases():
    # beta = 0 is plain ER; one step from t_prev = t0 is one plain ER step for
    # any beta; the noiseless truth is a fixed point of the accelerated map
    masks, t, g = small_problem(4, 4, K=4, P=3)
    op = ops.FFTOp(masks, 4, 4)
    I = ops.intensities(op, t)
    t0 = (g.standard_normal(t.shape) + 1j * g.standard_normal(t.shape)) / np.sqrt(2)
    plain = t0.copy()
    for _ in range(4):
        plain = rt.er_step(op, I, plain)
    assert np.max(np.abs(rt.er_accelerated(op, I, t0, 4, 0.0) - plain)) < 1e-13
    assert np.max(np.abs(rt.er_accelerated(op, I, t0, 1, 0.9) - rt.er_step(op, I, t0))) < 1e-13
    truth = t * np.exp(1j * 0.7)
    assert np.max(np.abs(rt.er_accelerated(op, I, truth, 10, 0.8) - truth)) < 1e-10


def test_accelerated_er_converges_faster_on_noiseless_rows():
    # Nesterov extrapolation of the ER step: with a positive factor the
    # noiseless 16x16 rows (K = 4, spectral start) reach the truth in fewer
    # iterations than plain ER; a negative factor slows it down
    n1 = n2 = 16
    N, K, P = n1 * n2, 4, 16
    masks = tm_synth.mask_phases(K, N, tm_synth.rng(5, 0))
    T = tm_synth.tm_iid(P, N, tm_synth.rng(5, 1))
    op = ops.FFTOp(masks, n1, n2)
    I = ops.intensities(op, T)
    v0 = tm_synth.random_start(P, N, np.ones(P), tm_synth.rng(5, 3))
    t0 = rt.spectral_start(op, I, v0, 40, momentum=0.98)
    f = {b: rt.fidelity(rt.er_accelerated(op, I, t0, 20, b), T) for b in (0.0, 0.8, -0.3)}
    assert f[0.8].min() > 0.95 and f[0.0].mean() < 0.95
    assert f[-0.3].mean() < f[0.0].mean() < f[0.8].mean()
    assert rt.fidelity(rt.er_accelerated(op, I, t0, 40, 0.8), T).min() > 0.999


def test_shifted_momentum_power_iteration():
    # M is PSD, so the rest of its spectrum lies in [0, lambda_2]: centring the
    # heavy-ball recurrence on that interval (lower = 0) reaches the top
    # eigenvector of the dense matrix (numpy.linalg.eigh) in fewer steps than
    # the symmetric interval; lower = -c is the unshifted recurrence
    masks, t, g = small_problem(4, 4, K=4, P=1, seed=23)
    d = ops.DenseOp(masks, 4, 4)
    I = ops.intensities(d, t)
    w = rt.spectral_weights(I, 3.0).reshape(-1)
    ev, V = np.linalg.eigh(d.A.conj().T @ (w[:, None] * d.A))
    assert ev[0] >= -1e-9 * ev[-1]
    c = ev[-2] / ev[-1]
    v0 = g.standard_normal((1, 16)) + 1j * g.standard_normal((1, 16))

    def overlap(v):
        return np.abs(np.vdot(V[:, -1], v[0])) ** 2 / np.vdot(v[0], v[0]).real

    a = rt.spectral_start(d, I, v0, 12, momentum=c)
    assert np.array_equal(a, rt.spectral_start(d, I, v0, 12, momentum=c, lower=-c))
    b = rt.spectral_start(d, I, v0, 12, momentum=c, lower=0.0)
    assert 1 - overlap(b) < 0.5 * (1 - overlap(a))
    assert overlap(rt.spectral_start(d, I, v0, 300, momentum=c, lower=0.0)) > 1 - 1e-10


def test_amplitude_gradient_finite_differences_and_er_identity():
    # the packed gradient of f_a = sum (sqrt(I) - |A t|)^2 against central
    # differences, and the identity grad f_a = 2 K N (t - ER(t)) that follows
    # from A^H A = K N I
    masks, t, g = small_problem(4, 4, K=3, P=2, seed=31)
    op = ops.FFTOp(masks, 4, 4)
    I = ops.intensities(op, t) * 1.3
    x = t + 0.3 * (g.standard_normal(t.shape) + 1j * g.standard_normal(t.shape))
    f, grad, _ = rt.amplitude_grad(op, I, x)
    for _ in range(3):
        v = g.standard_normal(t.shape) + 1j * g.standard_normal(t.shape)
        h = 1e-6
        fp, _, _ = rt.amplitude_grad(op, I, x + h * v)
        fm, _, _ = rt.amplitude_grad(op, I, x - h * v)
        fd = (fp - fm) / (2 * h)
        assert np.max(np.abs(fd - rt.rdot(grad, v))) <= 1e-6 * np.max(np.abs(fd))
    ident = 2 * op.K * op.N * (x - rt.er_step(op, I, x))
    assert np.max(np.abs(grad - ident)) <= 1e-10 * np.max(np.abs(grad))


def test_amplitude_line_search_picks_the_best_decreasing_trial():
    masks, t, g = small_problem(4, 4, K=4, P=3, seed=32)
    op = ops.FFTOp(masks, 4, 4)
    I = ops.intensities(op, t)
    x = t + 0.5 * (g.standard_normal(t.shape) + 1j * g.standard_normal(t.shape))
    f0, grad, y = rt.amplitude_grad(op, I, x)
    for d in (-grad / (2 * op.K * op.N), grad):  # a descent direction and an ascent one
        a = rt.amplitude_step(I, y, op.forward(d))
        fa = np.array([rt.amplitude_grad(op, I, x + s * d)[0] for s in rt.AMP_STEPS])  # [steps, P]
        for p in range(3):
            if a[p] == 0:
                assert np.all(fa[:, p] >= f0[p])
            else:
                fb = rt.amplitude_grad(op, I[p:p + 1], x[p:p + 1] + a[p] * d[p:p + 1])[0][0]
                assert fb < f0[p] and fb <= fa[:, p].min() + 1e-12 * f0[p]


def test_amplitude_lbfgs_monotone_and_recovers():
    n1 = n2 = 16
    N, K, P = n1 * n2, 4, 16
    masks = tm_synth.mask_phases(K, N, tm_synth.rng(5, 0))
    T = tm_synth.tm_iid(P, N, tm_synth.rng(5, 1))
    op = ops.FFTOp(masks, n1, n2)
    I = ops.intensities(op, T)
    v0 = tm_synth.random_start(P, N, np.ones(P), tm_synth.rng(5, 3))
    t0 = rt.spectral_start(op, I, v0, 40, momentum=0.98)
    t, hist = rt.lbfgs_amplitude(op, I, t0, 30)
    assert np.all(np.diff(hist, axis=0) <= 1e-12 * hist[0])
    assert rt.fidelity(t, T).min() > 0.999
    # its first step from an empty history is an error-reduction step when the unit trial wins
    t1, _ = rt.lbfgs_amplitude(op, I, t0, 1)
    f0, g0, y0 = rt.amplitude_grad(op, I, t0)
    a = rt.amplitude_step(I, y0, op.forward(-g0 / (2 * K * N)))
    assert np.allclose(t1, t0 + a[:, None] * (-g0 / (2 * K * N)))


def test_matrix_operator_gradient_matches_probing_form():
    # the dense operator with Q = A reproduces the structured gradient, and
    # with a random-phase Q its gradient passes central differences
    masks, t, g = small_problem(4, 4, K=3, P=2, seed=41)
    d = ops.DenseOp(masks, 4, 4)
    I = ops.intensities(d, t).reshape(2, -1) * 1.1
    mo = ops.MatrixOp(d.A)
    f1, g1, _ = rt.intensity_grad(mo, I, t + 0.2)
    f2, g2, _ = rt.intensity_grad(d, I.reshape(2, 3, 16), t + 0.2)
    assert np.allclose(f1, f2, rtol=1e-12) and np.allclose(g1, g2, rtol=1e-11, atol=1e-9)
    Q = tm_synth.random_phase_matrix(40, 16, tm_synth.rng(41, 7))
    mq = ops.MatrixOp(Q)
    Iq = np.abs(mq.forward(t)) ** 2
    x = t + 0.3
    f, grad, _ = rt.intensity_grad(mq, Iq, x)
    v = g.standard_normal(t.shape) + 1j * g.standard_normal(t.shape)
    fp = rt.intensity_grad(mq, Iq, x + 1e-6 * v)[0]
    fm = rt.intensity_grad(mq, Iq, x - 1e-6 * v)[0]
    assert np.max(np.abs((fp - fm) / 2e-6 - rt.rdot(grad, v))) <= 1e-5 * np.max(np.abs(fp))


def test_cyclic_er_substep_is_the_nearest_feasible_point():
    # one mask (K = 1): the update lands on {t : |F(psi t)|^2 = I} and is closer
    # to the input than any other point of that set (brute force over random
    # phases of the feasible spectrum, and over small phase perturbations of the
    # result itself)
    n1, n2 = 4, 4
    N = n1 * n2
    g = np.random.default_rng(41)
    psi = np.exp(2j * np.pi * g.random((1, N)))
    t = (g.standard_normal((1, N)) + 1j * g.standard_normal((1, N))) / np.sqrt(2)
    I = np.abs(g.standard_normal((1, 1, N))) * 3.0
    tp = rt.er_cyclic(psi, n1, n2, I, t, 1)
    F = ops.dft2_matrix(n1, n2)
    y = F @ (psi[0] * tp[0])
    assert np.max(np.abs(np.abs(y) ** 2 - I.reshape(N))) < 1e-12
    d0 = np.linalg.norm(tp - t)
    Finv = np.conj(F).T / N
    for _ in range(2000):
        th = np.exp(2j * np.pi * g.random(N))
        cand = np.conj(psi[0]) * (Finv @ (np.sqrt(I.reshape(N)) * th))
        assert np.linalg.norm(cand - t[0]) >= d0 - 1e-12
    ph = np.angle(y)
    for _ in range(200):
        cand = np.conj(psi[0]) * (Finv @ (np.sqrt(I.reshape(N)) * np.exp(1j * (ph + 0.05 * g.standard_normal(N)))))
        assert np.linalg.norm(cand - t[0]) >= d0 - 1e-12


def test_cyclic_er_fixed_point_two_mask_monotone_and_recovery():
    n1 = n2 = 8
    N, P = n1 * n2, 6
    masks = tm_synth.mask_phases(4, N, tm_synth.rng(42, 0))
    T = tm_synth.tm_iid(P, N, tm_synth.rng(42, 1))
    op = ops.FFTOp(masks, n1, n2)
    I = ops.intensities(op, T)
    # the noiseless truth, with any row phase, is a fixed point of a sweep
    truth = T * np.exp(1j * np.linspace(0, 3, P))[:, None]
    assert np.max(np.abs(rt.er_cyclic(masks, n1, n2, I, truth, 3) - truth)) < 1e-12
    # two sets (K = 2): alternating exact projections never lengthen the step
    # (the previous iterate lies in the set projected onto next)
    g = np.random.default_rng(43)
    t = (g.standard_normal((P, N)) + 1j * g.standard_normal((P, N))) / np.sqrt(2)
    I2 = I[:, :2]
    steps = []
    for k in range(30):
        tn = rt.er_cyclic(masks[k % 2: k % 2 + 1], n1, n2, I2[:, k % 2: k % 2 + 1], t, 1)
        steps.append(np.linalg.norm(tn - t, axis=1))
        t = tn
    steps = np.array(steps)
    assert np.all(steps[2:] <= steps[1:-1] * (1 + 1e-12) + 1e-12)
    # noiseless recovery from the spectral start (fidelity 0.9999, Sec. 2.2 data)
    v0 = tm_synth.random_start(P, N, np.ones(P), tm_synth.rng(42, 3))
    t0 = rt.spectral_start(op, I, v0, 40, momentum=0.98)
    assert rt.fidelity(rt.er_cyclic(masks, n1, n2, I, t0, 60), T).min() > 0.9999


def test_cyclic_er_sweep_sums_at_a_fixed_point_and_single_mask():
    # at the noiseless truth every term vanishes; with one mask the sums are
    # those of the start, computed by loops over the dense DFT
    n1, n2 = 4, 8
    N, P = n1 * n2, 3
    masks = tm_synth.mask_phases(3, N, tm_synth.rng(44, 0))
    T = tm_synth.tm_iid(P, N, tm_synth.rng(44, 1))
    I = ops.intensities(ops.FFTOp(masks, n1, n2), T)
    sa, si = rt.er_cyclic_sweep_sums(masks, n1, n2, I, T)
    assert np.max(sa) < 1e-20 and np.max(si) < 1e-18
    g = np.random.default_rng(45)
    t = (g.standard_normal((P, N)) + 1j * g.standard_normal((P, N))) / np.sqrt(2)
    sa1, si1 = rt.er_cyclic_sweep_sums(masks[:1], n1, n2, I[:, :1], t)
    F = ops.dft2_matrix(n1, n2)
    for p in range(P):
        y = F @ (masks[0] * t[p])
        ea = sum((np.sqrt(I[p, 0, k]) - abs(y[k])) ** 2 for k in range(N))
        ei = sum((I[p, 0, k] - abs(y[k]) ** 2) ** 2 for k in range(N))
        assert abs(sa1[p] - ea) < 1e-10 * ea and abs(si1[p] - ei) < 1e-10 * ei


def test_cyclic_er_needs_fewer_sweeps_than_parallel_er():
    # from the same spectral start on noiseless 16 x 16 rows, a cyclic sweep
    # (K projections in turn) gains more fidelity than a parallel ER step
    # (the average of the K projections)
    n1 = n2 = 16
    N, K, P = n1 * n2, 4, 12
    masks = tm_synth.mask_phases(K, N, tm_synth.rng(46, 0))
    T = tm_synth.tm_iid(P, N, tm_synth.rng(46, 1))
    op = ops.FFTOp(masks, n1, n2)
    I = ops.intensities(op, T)
    v0 = tm_synth.random_start(P, N, np.ones(P), tm_synth.rng(46, 3))
    t0 = rt.spectral_start(op, I, v0, 40, momentum=0.98)
    par = t0.copy()
    for _ in range(5):
        par = rt.er_step(op, I, par)
    cyc = rt.er_cyclic(masks, n1, n2, I, t0, 5)
    assert rt.fidelity(cyc, T).mean() > rt.fidelity(par, T).mean()


def _dense_M(masks, n1, n2, I, tau):
    A = ops.probing_matrix(masks, n1, n2)
    w = rt.spectral_weights(I, tau)
    return [np.conj(A).T @ (w[p].reshape(-1)[:, None] * A) for p in range(I.shape[0])]


def test_lanczos_start_equals_top_eigenvector_of_dense_M():
    # with k = N steps the Krylov space is everything: the Ritz vector is the
    # top eigenvector of the dense A^H diag(w) A (numpy eigh), up to phase
    n1, n2, K, P = 2, 4, 4, 3
    N = n1 * n2
    masks, t, g = small_problem(n1, n2, K=K, P=P, seed=51)
    op = ops.FFTOp(masks, n1, n2)
    I = ops.intensities(op, t)
    v0 = (g.standard_normal((P, N)) + 1j * g.standard_normal((P, N))) / np.sqrt(2)
    tl = rt.spectral_lanczos(op, I, v0, N, tau=3.0)
    Ms = _dense_M(masks, n1, n2, I, 3.0)
    for p in range(P):
        ev, vec = np.linalg.eigh(Ms[p])
        top = vec[:, -1]
        c = abs(np.vdot(top, tl[p])) / np.linalg.norm(tl[p])
        assert c > 1 - 1e-9
        assert abs(np.linalg.norm(tl[p]) ** 2 - I[p].sum() / (K * N)) < 1e-9 * I[p].sum()


def test_lanczos_basis_is_orthonormal_and_tridiagonalises_M():
    # exact-arithmetic Lanczos facts on a small problem (few steps, FP64):
    # V^H V = I and V^H M V = T (alpha on the diagonal, beta beside it);
    # the top Ritz value grows with k and stays below lambda_max; one step
    # returns the normalised seed
    n1, n2, K, P = 4, 4, 4, 2
    N = n1 * n2
    masks, t, g = small_problem(n1, n2, K=K, P=P, seed=52)
    op = ops.FFTOp(masks, n1, n2)
    I = ops.intensities(op, t)
    v0 = (g.standard_normal((P, N)) + 1j * g.standard_normal((P, N))) / np.sqrt(2)
    k = 6
    _, al, be, V = rt.spectral_lanczos(op, I, v0, k, tau=3.0, basis=True)
    Ms = _dense_M(masks, n1, n2, I, 3.0)
    for p in range(P):
        Vp = V[:k, p, :].T
        assert np.max(np.abs(np.conj(Vp).T @ Vp - np.eye(k))) < 1e-10
        Tm = np.diag(al[p]) + np.diag(be[p, :-1], 1) + np.diag(be[p, :-1], -1)
        assert np.max(np.abs(np.conj(Vp).T @ Ms[p] @ Vp - Tm)) < 1e-9 * np.max(np.abs(Tm))
        lam = np.linalg.eigvalsh(Ms[p])[-1]
        ritz = [np.linalg.eigvalsh(Tm[:j, :j])[-1] for j in range(1, k + 1)]
        assert all(ritz[j] <= ritz[j + 1] + 1e-12 * lam for j in range(k - 1)) and ritz[-1] <= lam * (1 + 1e-12)
    t1 = rt.spectral_lanczos(op, I, v0, 1, tau=3.0)
    ref = v0 / np.linalg.norm(v0, axis=1)[:, None] * np.sqrt(I.reshape(P, -1).sum(axis=1) / (K * N))[:, None]
    assert np.max(np.abs(t1 - ref)) < 1e-12


def test_lanczos_start_beats_power_iteration_at_equal_steps():
    # same number of operator applications: the Lanczos Ritz vector is closer
    # to the top eigenvector than plain power iteration's iterate
    n1 = n2 = 8
    N, K, P = n1 * n2, 4, 6
    masks = tm_synth.mask_phases(K, N, tm_synth.rng(53, 0))
    T = tm_synth.tm_iid(P, N, tm_synth.rng(53, 1))
    op = ops.FFTOp(masks, n1, n2)
    I = ops.intensities(op, T)
    v0 = tm_synth.random_start(P, N, np.ones(P), tm_synth.rng(53, 3))
    Ms = _dense_M(masks, n1, n2, I, 3.0)
    tl = rt.spectral_lanczos(op, I, v0, 8, tau=3.0)
    tp = rt.spectral_start(op, I, v0, 8, tau=3.0)
    for p in range(P):
        top = np.linalg.eigh(Ms[p])[1][:, -1]
        cl = abs(np.vdot(top, tl[p])) / np.linalg.norm(tl[p])
        cp = abs(np.vdot(top, tp[p])) / np.linalg.norm(tp[p])
        assert cl >= cp - 1e-12
