"""Pins of the FP64 phase-offset oracle (Sec. 2.3): operator equality,
closed forms of the angular-spectrum model, finite differences, noiseless
recovery. CPU only."""
import numpy as np
import pytest

import tm_synth
from oracle import defocus as df
from oracle.operators import dft_matrix

LAM = 1.0
PS = 0.5  # field pixel = lambda / 2


def setup(nf=8, P=20, N=12, Nd=5, NA=0.3, z=20.0, seed=3, dense=False):
    g = np.random.default_rng(seed)
    pix = np.sort(g.choice(nf * nf, P, replace=False))
    tm_est = g.standard_normal((P, N)) + 1j * g.standard_normal((P, N))
    theta = np.exp(2j * np.pi * g.random((Nd, N)))
    return df.DefocusModel(tm_est, theta, pix, nf, nf, LAM, PS, NA, z, dense=dense), g


def test_frequencies_are_numpy_fftfreq():
    for n in (1, 2, 5, 8, 16):
        assert np.allclose(df.freqs(n, 0.7), np.fft.fftfreq(n, 0.7))


def test_fft_model_equals_dense_matrices():
    m_fft, g = setup(nf=8, dense=False)
    m_dense, _ = setup(nf=8, dense=True)
    u = np.exp(1j * g.random(m_fft.c.shape[1]) * 6)
    a1, a2 = m_fft.forward(u), m_dense.forward(u)
    assert np.max(np.abs(a1 - a2)) < 1e-12 * np.max(np.abs(a1))
    v = g.standard_normal(a1.shape) + 1j * g.standard_normal(a1.shape)
    b1, b2 = m_fft.adjoint(v), m_dense.adjoint(v)
    assert np.max(np.abs(b1 - b2)) < 1e-12 * np.max(np.abs(b1))
    # adjoint identity
    lhs = np.vdot(a1, v)
    rhs = np.vdot(u, m_fft.adjoint(v))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_zero_defocus_is_fourier_interpolation():
    # at z = 0 a field band-limited by the pupil is interpolated exactly:
    # the even samples of the doubled grid equal the field / 2 (unitary K1, K2)
    nf = 16
    h, pupil = df.pupil_kernel(nf, nf, PS, LAM, 0.6, 0.0)
    g = np.random.default_rng(1)
    spec = (g.standard_normal((nf, nf)) + 1j * g.standard_normal((nf, nf))) * pupil
    field = np.fft.ifft2(spec)
    pix = np.arange(nf * nf)
    mdl = df.DefocusModel(np.diag(field.ravel()), np.ones((1, nf * nf)), pix, nf, nf, LAM, PS, 0.6, 0.0)
    out = mdl.forward(np.ones(nf * nf))[0]
    assert np.max(np.abs(out[::2, ::2] - field / 2)) < 1e-12 * np.max(np.abs(field))


def test_forward_then_backward_propagation_is_identity_on_band():
    h1, pupil = df.pupil_kernel(16, 16, PS, LAM, 0.3, 7.5)
    h2, _ = df.pupil_kernel(16, 16, PS, LAM, 0.3, -7.5)
    assert np.allclose(h1 * h2, pupil.astype(float), atol=1e-14)
    assert np.allclose(np.abs(h1), pupil.astype(float), atol=1e-14)


def test_pupil_includes_boundary_and_zeroes_nyquist():
    # a frequency exactly at NA / lambda is inside the pupil (the paper's <=)
    n = 10
    u = df.freqs(n, PS)
    NA = LAM * abs(u[2])
    _, pupil = df.pupil_kernel(n, n, PS, LAM, NA, 1.0)
    assert pupil[2, 0] and pupil[0, 2]
    for nf in (32, 64):
        _, p = df.pupil_kernel(nf, nf, PS, LAM, 0.3, 20.0)
        assert not p[nf // 2, :].any() and not p[:, nf // 2].any()


def test_phase_gradient_matches_finite_differences():
    mdl, g = setup(nf=8, P=10, N=8, Nd=4)
    phi_true = g.random(10) * 2 * np.pi
    Id = mdl.images(phi_true) + 0.05 * g.random((4, 16, 16))
    phi = phi_true + 0.3 * g.standard_normal(10)
    f0, grad = mdl.objective(Id, phi)
    h = 1e-6
    num = np.array([(mdl.objective(Id, phi + h * e)[0] - mdl.objective(Id, phi - h * e)[0]) / (2 * h)
                    for e in np.eye(10)])
    assert np.max(np.abs(num - grad)) < 1e-6 * np.max(np.abs(grad))
    # equals the paper's real(-4 diag(-j e^{-j phi}) sum A^H diag(A u) r) form
    u = np.exp(1j * phi)
    a = mdl.forward(u)
    w = mdl.adjoint(a * (Id - np.abs(a) ** 2))
    paper = np.real(-4 * (-1j * np.exp(-1j * phi)) * w)
    assert np.allclose(paper, grad, rtol=1e-12, atol=1e-12 * np.max(np.abs(grad)))


def test_constant_phase_invariance():
    mdl, g = setup()
    phi = g.random(20)
    Id = mdl.images(phi)
    assert np.allclose(mdl.images(phi + 1.234), Id, rtol=1e-12, atol=1e-12 * Id.max())


def test_noiseless_offsets_recovered():
    # TM_true = diag(e^{j phi}) TM_est; from phi = 0 L-BFGS recovers phi up to a constant
    # field band-limited to 0.6 of Nyquist, pupil NA 0.6 at ps = lambda / 2
    nf, P, N, Nd = 16, 40, 24, 12
    g = tm_synth.rng(42, 4)
    pix = tm_synth.nearest_pixels(nf, P)
    tm_true = tm_synth.speckle_tm(N, nf, 0.6, pix, tm_synth.rng(42, 1))
    phi_true = tm_synth.offsets(P, tm_synth.rng(42, 5))
    tm_est = np.exp(-1j * phi_true)[:, None] * tm_true
    theta = tm_synth.defocus_phases(Nd, N, g)
    mdl = df.DefocusModel(tm_est, theta, pix, nf, nf, LAM, PS, 0.6, 20 * LAM)
    Id = mdl.images(phi_true)
    phi, hist = df.lbfgs_phase(mdl, Id, np.zeros(P), 200)
    err = df.circular_offset_error(phi, phi_true)
    assert np.max(np.abs(err)) < 1e-8, np.max(np.abs(err))
    assert np.all(np.diff(hist) <= 0)


def test_line_search_postconditions():
    # The first direction is -sqrt(P) g/||g||. Replaying the first iteration's
    # trials on the objective evaluated afresh: the accepted step satisfies
    # Armijo; a step that grew stopped when a doubled trial was no better or the
    # curvature condition held (or at the cap); a halved step is the first trial
    # that satisfies Armijo.
    nf, P, N, Nd = 16, 40, 24, 12
    pix = tm_synth.nearest_pixels(nf, P)
    tm_true = tm_synth.speckle_tm(N, nf, 0.6, pix, tm_synth.rng(43, 1))
    phi_true = tm_synth.offsets(P, tm_synth.rng(43, 5))
    tm_est = np.exp(-1j * phi_true)[:, None] * tm_true
    theta = tm_synth.defocus_phases(Nd, N, tm_synth.rng(43, 4))
    mdl = df.DefocusModel(tm_est, theta, pix, nf, nf, LAM, PS, 0.6, 20 * LAM)
    Id = tm_synth.poisson_counts(mdl.images(phi_true), 1e4, tm_synth.rng(43, 6))
    for scale in (1.0, 1e-3, 30.0):  # first-step sizes that need no change, doublings, halvings
        phi0 = np.zeros(P)
        trace = []
        m2 = df.DefocusModel(tm_est, theta, pix, nf, nf, LAM, PS, 0.6, 20 * LAM)
        m2.objective = (lambda Idv, x, s=scale: (lambda fg: (fg[0], fg[1] * s))(mdl.objective(Idv, phi0 + x * s)))
        _, hist = df.lbfgs_phase(m2, Id, np.zeros(P), 1, trace=trace)
        f0, g0 = m2.objective(Id, np.zeros(P))
        d = -np.sqrt(P) * g0 / np.linalg.norm(g0)
        slope = g0 @ d
        steps = [t[0] for t in trace]
        assert steps[0] == 1.0
        grew = len(steps) > 1 and steps[1] == 2.0
        if grew:
            kept = [t for t in trace if t[3]]
            a_acc = kept[-1][0]
            f_acc, g_acc = m2.objective(Id, a_acc * d)
            last = trace[-1]
            assert (not last[3]) or g_acc @ d >= 0.9 * slope or len(steps) == 21
        else:
            a_acc = steps[-1]
            assert all(s2 == 0.5 * s1 for s1, s2 in zip(steps, steps[1:]))
            f_acc, _ = m2.objective(Id, a_acc * d)
            for a_rej in steps[:-1]:
                assert m2.objective(Id, a_rej * d)[0] > f0 + 1e-4 * a_rej * slope
        assert f_acc <= f0 + 1e-4 * a_acc * slope
        assert np.isclose(hist[1], f_acc, rtol=1e-13)
        print("scale", scale, "trials", steps)
