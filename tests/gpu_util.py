"""Helpers shared by the GPU tests: seeded problems (tm_synth) with expected
values from the FP64 oracle, and device transfer."""
import numpy as np
import torch

import tm_synth
from oracle import operators as ops


def dev():
    return torch.device("cuda:0")


def c64(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex64)).to(dev())


def f32(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev())


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def problem(n1, n2, K, P, cfg=900, noise=None, speckle=False):
    """masks, TM rows, intensities (FP64; Poisson noise at `noise` mean photons if given)."""
    N = n1 * n2
    masks = tm_synth.mask_phases(K, N, tm_synth.rng(cfg, 0))
    T = tm_synth.tm_iid(P, N, tm_synth.rng(cfg, 1))
    op = ops.FFTOp(masks, n1, n2)
    I = ops.intensities(op, T)
    if noise:
        I = tm_synth.poisson_counts(I, noise, tm_synth.rng(cfg, 2))
    return masks, T, I, op


def rounded(masks, T, I):
    """FP32-rounded copies (what the GPU receives), as FP64 arrays."""
    return (masks.astype(np.complex64).astype(np.complex128), T.astype(np.complex64).astype(np.complex128),
            I.astype(np.float32).astype(np.float64))


def oracle_intensities(masks, T, n1, n2, chunk=128):
    """|A t|^2 of every row in FP64 by the oracle's FFT form, from the
    FP32-rounded masks and rows the GPU receives (row chunks bound the memory)."""
    m = np.asarray(masks).astype(np.complex64).astype(np.complex128)
    op = ops.FFTOp(m, n1, n2)
    T = np.asarray(T)
    out = np.empty((T.shape[0], m.shape[0], n1 * n2), dtype=np.float64)
    for i0 in range(0, T.shape[0], chunk):
        out[i0:i0 + chunk] = ops.intensities(op, T[i0:i0 + chunk].astype(np.complex64).astype(np.complex128))
    return out


def device_intensities(I, bf16=False):
    """FP64 intensities as the GPU's input (FP32, or BF16 rounded to nearest
    even on the host), and the same values back as FP64 for the oracle."""
    t = torch.from_numpy(np.ascontiguousarray(I, dtype=np.float32))
    if bf16:
        t = t.to(torch.bfloat16)
    return t.to(dev()), t.to(torch.float64).numpy()
