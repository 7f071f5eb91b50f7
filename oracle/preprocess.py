"""Preprocessing of the measured intensity images, FP64 (test infrastructure only).

Follows Sec. 2.2 (the paragraph after Algorithm 1, and the experiment in
Sec. 3): the camera images are half-sampled, a binary fiber mask keeping
99.9 % of the total intensity is derived from them, and only the pixels
inside the mask become optimisation problems, each with its vector of
K N intensities (one per probing pattern, i.e. per image).

Readings where the paper is silent:
  * "pixels of the odd indexes" counts from 1 (the first pixel is index 1),
    so the kept pixels are the 0-based even rows and columns:
    stack[:, 0::2, 0::2].
  * The mask is the smallest set of half-sampled pixels whose summed
    intensity (over all images) reaches frac = 0.999 of the total: pixels
    are taken by decreasing summed intensity, ties by increasing raster
    index, until the running sum first reaches frac * total. A stack with
    zero total intensity has an empty mask.
  * Pixel rows are returned in increasing raster order of the half-sampled
    grid, and each row's measurements in image order (the row order of A,
    mask-major).
"""
from __future__ import annotations

import numpy as np


def half_sample(stack: np.ndarray) -> np.ndarray:
    """[n_img][H][W] -> [n_img][H/2][W/2]: the 1-based odd rows and columns."""
    return stack[:, 0::2, 0::2]


def energy(stack: np.ndarray) -> np.ndarray:
    """Summed intensity of every half-sampled pixel over all images, FP64,
    flattened in raster order."""
    h = half_sample(np.asarray(stack)).astype(np.float64)
    return h.sum(axis=0).reshape(-1)


def fiber_mask(E: np.ndarray, frac: float = 0.999) -> np.ndarray:
    """Raster indices (ascending) of the smallest brightest-first pixel set
    whose summed intensity reaches frac of the total."""
    E = np.asarray(E, dtype=np.float64)
    total = E.sum()
    if not total > 0:
        return np.zeros(0, dtype=np.int64)
    order = np.argsort(-E, kind="stable")
    running = np.cumsum(E[order])
    count = int(np.searchsorted(running, frac * total, side="left")) + 1
    return np.sort(order[:min(count, E.size)])


def gather_rows(stack: np.ndarray, pix: np.ndarray) -> np.ndarray:
    """[P][n_img]: for each masked pixel, its intensity in every image."""
    h = half_sample(np.asarray(stack))
    return h.reshape(h.shape[0], -1)[:, pix].T.copy()
