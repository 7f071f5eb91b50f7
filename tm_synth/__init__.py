"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module draws random numbers and builds test inputs; it holds none of
the retrieval method's arithmetic (no probing operator, no loss, no solver).
Every stream is ``numpy.random.default_rng([config_id, stream])`` so that a
(config, stream) pair always produces the same values.

Streams: 0 masks, 1 TM, 2 intensity noise, 3 start vector, 4 defocus input
phases, 5 defocus noise, 6 network init / shuffling.

Where the paper's data are measured (holography or Maxwell-simulated TMs,
camera stacks), these generators stand in with the same shapes: mask phases
i.i.d. uniform (Sec. 2.2, the probing-matrix design), TM rows i.i.d.
circular Gaussian or band-limited speckle, Poisson shot noise.
"""
from __future__ import annotations

import numpy as np

STREAM_MASKS, STREAM_TM, STREAM_NOISE, STREAM_START, STREAM_DEFOCUS, STREAM_DNOISE, STREAM_NET = range(7)


def rng(config_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(config_id), int(stream)])


def mask_phases(K: int, N: int, g: np.random.Generator) -> np.ndarray:
    """K random phase masks: unit-modulus complex128 [K, N], phases U[0, 2pi)."""
    return np.exp(2j * np.pi * g.random((K, N)))


def tm_iid(P: int, N: int, g: np.random.Generator) -> np.ndarray:
    """P x N circular complex Gaussian CN(0, 1) rows, complex128."""
    return (g.standard_normal((P, N)) + 1j * g.standard_normal((P, N))) / np.sqrt(2.0)


def nearest_pixels(grid: int, count: int) -> np.ndarray:
    """Raster indices of the `count` pixels of a grid x grid image nearest to
    the centre (grid//2, grid//2); ties broken by raster index. Stands in for
    the binary fiber mask (a disk of pixels)."""
    c = grid // 2
    yy, xx = np.meshgrid(np.arange(grid), np.arange(grid), indexing="ij")
    d2 = ((yy - c) ** 2 + (xx - c) ** 2).ravel()
    order = np.lexsort((np.arange(grid * grid), d2))
    return np.sort(order[:count]).astype(np.int64)


def speckle_tm(N: int, grid: int, pupil_frac: float, pixels: np.ndarray,
               g: np.random.Generator, chunk: int = 1024) -> np.ndarray:
    """Band-limited speckle TM of shape [len(pixels), N], complex128.

    Each column is white CN(0,1) on a grid x grid output plane, low-passed by
    a circular pupil whose radius is `pupil_frac` of the grid Nyquist
    frequency, and sampled at `pixels`. Columns are independent, so each row
    is i.i.d. across columns; rows are spatially correlated. Scaled so that
    the mean power per entry is 1.
    """
    f = np.fft.fftfreq(grid)  # cycles/sample, Nyquist = 0.5
    fy, fx = np.meshgrid(f, f, indexing="ij")
    pupil = (np.sqrt(fy ** 2 + fx ** 2) <= pupil_frac * 0.5).astype(np.float64)
    out = np.empty((len(pixels), N), dtype=np.complex128)
    for c0 in range(0, N, chunk):
        c1 = min(N, c0 + chunk)
        w = (g.standard_normal((c1 - c0, grid, grid)) + 1j * g.standard_normal((c1 - c0, grid, grid))) / np.sqrt(2.0)
        fld = np.fft.ifft2(np.fft.fft2(w) * pupil)
        out[:, c0:c1] = fld.reshape(c1 - c0, grid * grid)[:, pixels].T
    out /= np.sqrt(np.mean(np.abs(out) ** 2))
    return out


def random_start(P: int, N: int, sigma2: np.ndarray, g: np.random.Generator) -> np.ndarray:
    """Random start rows t0 ~ CN(0, sigma2[p]) (caller chooses sigma2)."""
    s = np.sqrt(np.asarray(sigma2, dtype=np.float64) / 2.0)[:, None]
    return (g.standard_normal((P, N)) + 1j * g.standard_normal((P, N))) * s


def poisson_counts(clean: np.ndarray, mean_photons: float, g: np.random.Generator) -> np.ndarray:
    """Shot noise: scale clean intensities so their global mean is
    `mean_photons`, draw Poisson counts, scale back. float64, same shape."""
    s = mean_photons / float(np.mean(clean))
    return g.poisson(clean * s).astype(np.float64) / s


def defocus_phases(Nd: int, N: int, g: np.random.Generator) -> np.ndarray:
    """Nd random-phase incident fields e^{j theta_n}, unit modulus [Nd, N]."""
    return np.exp(2j * np.pi * g.random((Nd, N)))


def offsets(P: int, g: np.random.Generator) -> np.ndarray:
    """Per-row phase offsets phi in [0, 2pi) (for building TM_est = diag(e^{-j phi}) TM_true)."""
    return 2 * np.pi * g.random(P)


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest even); returns uint16 bit patterns."""
    f = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    rounding = ((f >> 16) & 1) + np.uint32(0x7FFF)
    return ((f + rounding) >> 16).astype(np.uint16)


def from_bf16_bits(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint32) << 16).view(np.float32)


def fiber_disk(H: int, W: int, radius: float) -> np.ndarray:
    """Boolean [H, W] disk centred on the image (the fiber core seen by the camera)."""
    y, x = np.mgrid[0:H, 0:W]
    return (y - (H - 1) / 2) ** 2 + (x - (W - 1) / 2) ** 2 <= radius ** 2


def camera_stack(n_img: int, H: int, W: int, radius: float, g: np.random.Generator, peak: float = 4000.0,
                 background: float = 0.05) -> np.ndarray:
    """uint16 [n_img, H, W] camera counts: exponential (speckle-like) intensities
    of mean peak/4 inside the fiber disk, Poisson background of mean
    `background` outside."""
    inside = fiber_disk(H, W, radius)
    speckle = np.minimum(g.exponential(peak / 4, size=(n_img, H, W)), 65535.0)
    bg = g.poisson(background, size=(n_img, H, W)).astype(np.float64)
    return np.where(inside[None], np.floor(speckle), bg).astype(np.uint16)


def random_phase_matrix(M: int, N: int, g: np.random.Generator) -> np.ndarray:
    """Dense probing matrix with i.i.d. uniform phases, unit modulus [M, N]
    (the prior-art random-phase probing)."""
    return np.exp(2j * np.pi * g.random((M, N)))
