"""Learned start at N = 1024 (32 x 32 modes), K = 4, one fixed mask set:
train on forward-model rows on the GPU, then compare on held-out rows with
the plain (spectral-start) method. Records the measured gain; asserts the
machinery (training lowers the loss, the fallback reaches fidelity 0.99)."""
import time

import numpy as np
import pytest
import torch

import paper_2302_13524_amd as tm
import tm_synth
from oracle import operators as ops
from oracle import retrieval as rt
from paper_2302_13524_amd import learned

from gpu_util import c64, dev, f32

pytestmark = pytest.mark.gpu


def test_learned_start_gain():
    ctx = tm.Context(0)
    n1 = n2 = 32
    N, K, P = 1024, 4, 512
    masks_np = tm_synth.mask_phases(K, N, tm_synth.rng(4, 0))
    masks = c64(masks_np)
    net = tm.MLP(K * N, 1024, 2 * N, seed=6)
    t0 = time.perf_counter()
    hist = learned.train(ctx, net, masks, n1, n2, rows=200_000, epochs=2, batch=512, lr=1e-3, seed=6,
                         log=lambda s: print(s, flush=True))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    # held-out rows (other seeds), Poisson 1e4
    T = tm_synth.tm_iid(P, N, tm_synth.rng(40, 1))
    I = ops.intensities(ops.FFTOp(masks_np, n1, n2), T)
    I = tm_synth.poisson_counts(I, 1e4, tm_synth.rng(40, 2)).astype(np.float32)
    It = f32(I)
    seed_rows = c64(tm_synth.random_start(P, N, I.reshape(P, -1).sum(1) / (K * N * N), tm_synth.rng(40, 3)))
    fid = lambda t: rt.fidelity(t.cpu().numpy().astype(np.complex128), T)
    f_learned = fid(tm.tm_mlp_start(ctx, net, It, K, N)).mean()
    f_random = fid(seed_rows).mean()
    # plain form: spectral start + ER to mean fidelity 0.99
    iters = 100

    def plain():
        t = seed_rows.clone()
        tm.tm_retrieve(ctx, masks, It, t, n1, n2, tm.retrieve_opts("er", iters=iters, start="spectral"))
        return t

    def learned_form():
        return learned.retrieve_with_fallback(ctx, net, masks, It, n1, n2, iters, seed_rows)

    tp = plain()
    tl, redone = learned_form()
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(3):
        plain()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - a) / 3
    a = time.perf_counter()
    for _ in range(3):
        learned_form()
    torch.cuda.synchronize()
    t_learned = (time.perf_counter() - a) / 3
    fp, fl = fid(tp).mean(), fid(tl).mean()
    print(f"train {train_s:.1f}s loss {hist}; start fidelity learned {f_learned:.5f} random {f_random:.5f}; "
          f"rows redone from the fallback {redone}/{P}; final fidelity plain {fp:.5f} learned {fl:.5f}; "
          f"wall plain {t_plain*1e3:.2f} ms learned {t_learned*1e3:.2f} ms")
    assert np.all(np.isfinite(hist)) and hist[-1] <= hist[0]
    assert fp >= 0.99 and fl >= 0.99
    ctx.close()
