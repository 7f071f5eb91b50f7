"""Learned start: training the weighting network on forward-model data and
installing its table (a driver around the library's network entry points).

The learned start proposes the weighting function T(x) of the spectral start
(tm_wnet_*): the start stays the top eigenvector of A^H diag(T(x)) A, found
by Lanczos steps, and only the weights are learned. (The library's other
network, tm_mlp_*, proposes start rows directly from a row's intensities; at
K = 4 its start is no better than a random one, a measured negative result
kept with its tests.)

Training rows are generated on the GPU: random TM rows CN(0, 1), their
intensities by the probing operator of Sec. 2.2 (Eq. probingmatrix), Poisson
shot noise at a given mean photon count. The retrieval from the learned
start, with the per-row fallback to the plain start where the FP64
acceptance residual stays above a threshold, is tm_retrieve_learned.
"""
from __future__ import annotations

import time

import torch

from . import tm_forward, tm_set_weight_table, tm_wnet_pretrain_step, tm_wnet_table, tm_wnet_train_step, weight_net


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
