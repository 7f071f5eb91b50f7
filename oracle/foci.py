"""Foci synthesis with a retrieved TM and their power ratio, FP64 (test
infrastructure only).

Follows Sec. 3 (the validation of the retrieved TM): the phase of the
conjugate of each retrieved row is displayed on the phase modulator, the
true system forms the output field, and a focus appears at that row's pixel
when the row is right. Its quality is the power ratio PR: the power in a
7 x 7 pixel window around the peak over the total power of the image.

Readings where the paper is silent:
  * The displayed pattern for row p is the unit-modulus u_p = exp(-j arg
    tm_est[p]) (phase-only modulation), and the output field at pixel q is
    sum_n tm_true[q][n] u_p[n]: the images live on the pixels of the TM rows
    (the masked pixels of the output grid), dark elsewhere.
  * The peak is the brightest pixel of the image (the first in raster order
    on ties); the window is the (2w+1) x (2w+1) block of grid pixels centred
    on it (w = 3: 7 x 7), clipped at the grid border; an image with no power
    has PR 0.
  * The paper's two exposures (a short one for the window, a long one scaled
    by 20 for the background) only extend the camera's range; in simulation
    both sums come from the same image.
  * The propagated TM at a defocus distance z (Sec. 4, 3-D foci) applies the
    free-space angular-spectrum propagation of Eq. angularspectrum (pupil
    NA, same kernel as the phase-correction model) to every column of the TM
    laid out on the output grid (rows outside the TM's pixels are zero), and
    keeps every grid pixel: TM_z [g1 g2][N].
"""
from __future__ import annotations

import numpy as np

from .defocus import pupil_kernel


def focus_patterns(tm_est: np.ndarray) -> np.ndarray:
    """u [P][N]: phase of the conjugate of each retrieved row, unit modulus."""
    return np.exp(-1j * np.angle(tm_est))


def focus_intensities(tm_true: np.ndarray, tm_est: np.ndarray) -> np.ndarray:
    """[P foci][P pixels]: |sum_n tm_true[q][n] u_p[n]|^2."""
    E = focus_patterns(tm_est) @ tm_true.T
    return np.abs(E) ** 2


def propagate_tm(tm: np.ndarray, pix: np.ndarray, g1: int, g2: int, lam: float, ps: float, NA: float,
                 z: float) -> np.ndarray:
    """TM_z [g1 g2][N]: each column on the g1 x g2 grid, propagated by z with
    the angular-spectrum kernel (fft2, times h, inverse fft2)."""
    P, N = tm.shape
    grid = np.zeros((g1 * g2, N), dtype=np.complex128)
    grid[pix] = tm
    cols = grid.T.reshape(N, g1, g2)
    h, _ = pupil_kernel(g1, g2, ps, lam, NA, z)
    out = np.fft.ifft2(np.fft.fft2(cols, axes=(1, 2)) * h[None], axes=(1, 2))
    return out.reshape(N, g1 * g2).T.copy()


def power_ratio(img: np.ndarray, pix: np.ndarray, g1: int, g2: int, w: int = 3):
    """(PR, peak raster index) of one focus image given on the pixels pix of a
    g1 x g2 grid."""
    grid = np.zeros(g1 * g2)
    grid[pix] = img
    total = grid.sum()
    if not total > 0:
        return 0.0, -1
    peak = int(np.argmax(grid))
    y, x = divmod(peak, g2)
    g = grid.reshape(g1, g2)
    sig = g[max(0, y - w):min(g1, y + w + 1), max(0, x - w):min(g2, x + w + 1)].sum()
    return float(sig / total), peak


def foci_power_ratios(tm_true: np.ndarray, tm_est: np.ndarray, pix: np.ndarray, g1: int, g2: int, w: int = 3):
    """PR and peak of the focus of every row of tm_est [Pf][N] (the patterns),
    with images over the rows of tm_true [G][N] at the pixels pix [G]."""
    F = focus_intensities(tm_true, tm_est)
    out = [power_ratio(F[p], pix, g1, g2, w) for p in range(F.shape[0])]
    return np.array([o[0] for o in out]), np.array([o[1] for o in out])
