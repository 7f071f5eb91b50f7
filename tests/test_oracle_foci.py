"""Pins of the foci / power-ratio oracle against closed forms. CPU only."""
import numpy as np

import tm_synth
from oracle import foci


def test_conjugate_phase_focus_at_its_pixel():
    # with the true row displayed in conjugate phase, the field at that row's
    # pixel is sum_n |tm_pn|, the largest any unit-modulus pattern can give
    T = tm_synth.tm_iid(12, 40, tm_synth.rng(990, 1))
    F = foci.focus_intensities(T, T)
    assert np.allclose(np.diag(F), np.sum(np.abs(T), axis=1) ** 2, rtol=1e-12)
    g = np.random.default_rng(3)
    for p in range(12):
        u = np.exp(2j * np.pi * g.random(40))
        assert abs(u @ T[p]) ** 2 <= F[p, p] * (1 + 1e-12)


def test_focus_ignores_a_row_phase():
    T = tm_synth.tm_iid(6, 30, tm_synth.rng(991, 1))
    est = T * np.exp(1j * np.linspace(0, 5, 6))[:, None]
    assert np.allclose(foci.focus_intensities(T, est), foci.focus_intensities(T, T), rtol=1e-12)


def test_power_ratio_closed_forms():
    g1, g2 = 16, 12
    pix = np.arange(g1 * g2)
    flat = np.ones(g1 * g2)
    # uniform image, peak at raster 0 (first on ties): window clipped to 4 x 4
    pr, peak = foci.power_ratio(flat, pix, g1, g2, 3)
    assert peak == 0 and abs(pr - 16 / (g1 * g2)) < 1e-15
    # all the power inside the window around an interior peak
    img = np.zeros(g1 * g2)
    img[7 * g2 + 6] = 5.0
    img[5 * g2 + 4] = 1.0
    img[9 * g2 + 9] = 2.0
    pr, peak = foci.power_ratio(img, pix, g1, g2, 3)
    assert peak == 7 * g2 + 6 and pr == 1.0
    img[0] = 8.0  # the corner becomes the peak; its clipped window holds only itself
    pr, peak = foci.power_ratio(img, pix, g1, g2, 3)
    assert peak == 0 and abs(pr - 8.0 / 16.0) < 1e-15
    assert foci.power_ratio(np.zeros(4), np.arange(4), 2, 2)[0] == 0.0


def test_power_ratio_on_a_pixel_subset_by_loops():
    g = np.random.default_rng(5)
    g1, g2 = 10, 9
    pix = np.sort(g.choice(g1 * g2, 40, replace=False))
    img = g.random(40)
    pr, peak = foci.power_ratio(img, pix, g1, g2, 2)
    grid = {int(q): v for q, v in zip(pix, img)}
    py, px = divmod(peak, g2)
    sig = sum(v for q, v in grid.items() if abs(q // g2 - py) <= 2 and abs(q % g2 - px) <= 2)
    assert abs(pr - sig / img.sum()) < 1e-14 and peak == pix[np.argmax(img)]


def _band_limited(g1, g2, N, NA, ps, lam, seed):
    # columns whose spectrum lies inside the pupil (so propagation is exact)
    from oracle.defocus import pupil_kernel
    _, pupil = pupil_kernel(g1, g2, ps, lam, NA, 0.0)
    g = np.random.default_rng(seed)
    spec = (g.standard_normal((N, g1, g2)) + 1j * g.standard_normal((N, g1, g2))) * pupil[None]
    return np.fft.ifft2(spec, axes=(1, 2)).reshape(N, g1 * g2).T.copy()


def test_propagation_identities():
    g1, g2, N, lam, ps, NA = 16, 8, 5, 1.0, 0.5, 0.6
    cols = _band_limited(g1, g2, N, NA, ps, lam, 7)      # [G][N] on every pixel
    pix = np.arange(g1 * g2)
    assert np.allclose(foci.propagate_tm(cols, pix, g1, g2, lam, ps, NA, 0.0), cols, atol=1e-12)
    a = foci.propagate_tm(cols, pix, g1, g2, lam, ps, NA, 3.0)
    b = foci.propagate_tm(a, pix, g1, g2, lam, ps, NA, 4.5)
    assert np.allclose(b, foci.propagate_tm(cols, pix, g1, g2, lam, ps, NA, 7.5), atol=1e-12)
    assert np.allclose(np.linalg.norm(a, axis=0), np.linalg.norm(cols, axis=0), rtol=1e-12)  # unitary in band
    back = foci.propagate_tm(a, pix, g1, g2, lam, ps, NA, -3.0)
    assert np.allclose(back, cols, atol=1e-12)


def test_plane_wave_takes_the_angular_spectrum_phase():
    # a grid plane wave of frequency (u, v) propagates by exp(j 2 pi / lambda sqrt(1 - lambda^2 (u^2 + v^2)) z)
    g1, g2, lam, ps, NA, z = 16, 16, 1.0, 0.5, 0.9, 2.5
    k1, k2 = 3, -2
    y, x = np.mgrid[0:g1, 0:g2]
    wave = np.exp(2j * np.pi * (k1 * y / g1 + k2 * x / g2)).reshape(-1, 1)
    out = foci.propagate_tm(wave, np.arange(g1 * g2), g1, g2, lam, ps, NA, z)
    u, v = k1 / (g1 * ps), k2 / (g2 * ps)
    phase = np.exp(1j * 2 * np.pi / lam * np.sqrt(1 - lam ** 2 * (u * u + v * v)) * z)
    assert np.allclose(out, wave * phase, atol=1e-12)
