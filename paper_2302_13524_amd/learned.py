"""Learned start: training on forward-model data and the start-with-fallback
retrieval (driver around the library's network entry points).

Two networks are here. The first proposes start rows directly from a row's
intensities (tm_mlp_*); at K = 4 its start is no better than a random one
(kept as a measured negative result). The second, the learned start that is
used, proposes the weighting function T(x) of the spectral start
(tm_wnet_*): the start stays the top eigenvector of A^H diag(T(x)) A, found
by Lanczos steps, and only the weights are learned.

Training pairs are generated on the GPU: random TM rows CN(0, 1) from a
seeded device generator, their intensities by tm_forward (the probing
operator of Sec. 2.2, Eq. probingmatrix), Poisson shot noise at a given
mean photon count. Every training step (features, three BF16 MFMA layers,
phase-invariant loss, backward, Adam) is one tm_mlp_train_step call.

The learned start is judged by the plain iteration: rows whose FP64
acceptance residual after the iterations stays above the flag threshold are
re-run from the fallback (truncated spectral) start.
"""
from __future__ import annotations

import time

import torch

from . import (MLP, TMError, decode_stats, retrieve_opts, tm_forward, tm_mlp_start, tm_mlp_train_step,
               tm_retrieve, tm_set_weight_table, tm_wnet_pretrain_step, tm_wnet_table, tm_wnet_train_step,
               weight_net)


def make_batch(ctx, masks, n1, n2, rows, gen, photons=1e4):
    """(I [rows, K, N] float32 with shot noise, t [rows, N] complex64)."""
    N = n1 * n2
    dev = masks.device
    t = torch.complex(torch.randn((rows, N), generator=gen, device=dev),
                      torch.randn((rows, N), generator=gen, device=dev)) * (0.5 ** 0.5)
    t = t.to(torch.complex64).contiguous()
    I = tm_forward(ctx, masks, t, n1, n2, intensity=True)
    if photons:
        scale = photons / I.mean()
        I = (torch.poisson(I * scale, generator=gen) / scale).contiguous()
    return I, t


def train(ctx, net: MLP, masks, n1, n2, rows=200_000, epochs=3, batch=512, lr=1e-3, seed=6, photons=1e4,
          log=None):
    """Train on `rows` fresh forward-model rows per epoch (generated per batch).
    Returns the mean training loss of each epoch."""
    K, N = masks.shape
    gen = torch.Generator(device=masks.device)
    gen.manual_seed(seed)
    loss = torch.empty((batch,), dtype=torch.float32, device=masks.device)
    net.sync(ctx)
    hist = []
    for ep in range(epochs):
        acc = torch.zeros((), dtype=torch.float64, device=masks.device)
        nb = max(1, rows // batch)
        t0 = time.perf_counter()
        for _ in range(nb):
            I, t = make_batch(ctx, masks, n1, n2, batch, gen, photons)
            tm_mlp_train_step(ctx, net, I, t, K, N, lr, loss)
            acc += loss.double().mean()
        hist.append(acc.item() / nb)
        if log:
            log(f"epoch {ep}: mean loss {hist[-1]:.5f} ({time.perf_counter() - t0:.2f}s)")
    return hist


def retrieve_with_fallback(ctx, net: MLP, masks, I, n1, n2, iters, seed_rows, spectral_iters=30,
                           spectral_momentum=0.98, rho_flag=1e-2, er_momentum=0.0, spectral_tau=3.0,
                           spectral_lower=None, method="er", start="spectral"):
    """Learned start -> `iters` iterations of the error-reduction `method` -> rows whose FP64
    residual exceeds rho_flag are redone from the spectral start (seeded with
    `seed_rows`). Returns (t, number of rows redone)."""
    K, N = masks.shape
    if I.dtype != torch.float32:
        raise TMError("the learned start reads float32 intensities")
    t = tm_mlp_start(ctx, net, I, K, N)
    raw = tm_retrieve(ctx, masks, I, t, n1, n2, retrieve_opts(method, iters=iters, start="given",
                                                              er_momentum=er_momentum))
    st = decode_stats(raw)
    bad = torch.nonzero(st.rho > rho_flag).flatten()
    if bad.numel():
        idx = bad.to(I.device)
        tb = seed_rows.index_select(0, idx).contiguous()
        Ib = I.index_select(0, idx).contiguous()
        tm_retrieve(ctx, masks, Ib, tb, n1, n2,
                    retrieve_opts(method, iters=iters, start=start, spectral_iters=spectral_iters,
                                  spectral_tau=spectral_tau, spectral_momentum=spectral_momentum,
                                  spectral_lower=spectral_lower, er_momentum=er_momentum))
        t.index_copy_(0, idx, tb)
    return t, int(bad.numel())


def train_weights(ctx, masks, n1, n2, steps=150, rows=128, power_steps=20, pretrain_steps=200, tau=3.0, nt=256,
                  xmax=16.0, lr=2e-4, pretrain_lr=2e-3, hidden=256, seed=6, photons=1e4, net=None, log=None):
    """Train the weighting network: a warm start that fits the plain
    truncation min(x, tau) on the table points, then `steps` training steps,
    each on `rows` fresh forward-model rows (CN(0, 1) rows, intensities by
    tm_forward with Poisson noise, random seeds), `power_steps` power
    iterations deep. Adam's step is kept small (2e-4): the power iteration
    follows the eigenvalue of largest magnitude, so a step that makes T(x)
    strongly negative near x = 0 flips it to the bottom of the spectrum,
    where the loss has no useful gradient (measured: 1e-3 collapses the
    fidelity to 0, 1e-4 and 3e-4 converge to the same table). Returns (net,
    per-step losses as a device tensor)."""
    dev = masks.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    net = net if net is not None else weight_net(hidden, device=dev, seed=seed)
    net.sync(ctx)
    loss = torch.empty((1,), dtype=torch.float32, device=dev)
    for _ in range(pretrain_steps):
        tm_wnet_pretrain_step(ctx, net, nt, xmax, tau, pretrain_lr, loss)
    hist = torch.empty((steps,), dtype=torch.float32, device=dev)
    N = n1 * n2
    t0 = time.perf_counter()
    for i in range(steps):
        I, t = make_batch(ctx, masks, n1, n2, rows, gen, photons)
        v0 = torch.complex(torch.randn((rows, N), generator=gen, device=dev),
                           torch.randn((rows, N), generator=gen, device=dev)).to(torch.complex64).contiguous()
        tm_wnet_train_step(ctx, net, masks, I, t, v0, n1, n2, power_steps, nt, xmax, lr, loss)
        hist[i:i + 1].copy_(loss)
    if log:
        torch.cuda.synchronize()
        log(f"weight network: {steps} steps in {time.perf_counter() - t0:.2f}s, loss {hist[:5].mean().item():.4f} "
            f"-> {hist[-5:].mean().item():.4f}")
    return net, hist


def install_weights(ctx, net, nt=256, xmax=16.0):
    """Evaluate the network on its table and hand the table to the context (TM_START_LEARNED)."""
    tab = tm_wnet_table(ctx, net, nt, xmax)
    tm_set_weight_table(ctx, tab, xmax)
    return tab
