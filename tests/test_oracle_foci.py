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
