"""GPU parity of the learned weighting of the spectral start (through the C
ABI) against its FP64 reference: the network's table, the power-iteration
training loss and its table gradient, a training step's parameter update,
the Lanczos start with a weight table, and the fallback to the plain start."""
import numpy as np
import pytest
import torch

import paper_2302_13524_amd as tm
import tm_synth
from oracle import learned_weights as lw
from oracle import mlp as omlp
from oracle import operators as ops
from oracle import retrieval as rt

from gpu_util import c64, dev, device_intensities, f32, oracle_intensities, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tm.Context(0)
    yield c
    c.close()


def bf16_round(x):
    return torch.as_tensor(np.asarray(x), dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()


def seeded_net(hidden=32, seed=11):
    g = np.random.default_rng(seed)
    p = omlp.init_params(lw.N_FEAT, hidden, 1, g)
    for k in ("b1", "b2", "b3"):
        p[k] = 0.05 * g.standard_normal(p[k].shape)
    for k in ("W1", "W2", "W3"):
        p[k] = bf16_round(p[k])  # the device multiplies BF16 copies of its FP32 masters
    net = tm.MLP(lw.N_FEAT, hidden, 1, weights=[(p["W1"], p["b1"]), (p["W2"], p["b2"]), (p["W3"], p["b3"])])
    return p, net


def data(n1, n2, P, cfg, K=4):
    N = n1 * n2
    masks = tm_synth.mask_phases(K, N, tm_synth.rng(cfg, 0))
    T = tm_synth.tm_iid(P, N, tm_synth.rng(cfg, 1)).astype(np.complex64)
    I64 = tm_synth.poisson_counts(oracle_intensities(masks, T, n1, n2), 1e4, tm_synth.rng(cfg, 2))
    v0 = tm_synth.random_start(P, N, np.ones(P), tm_synth.rng(cfg, 3)).astype(np.complex64)
    return masks, T, I64, v0


@pytest.mark.parametrize("nt,hidden", [(256, 32), (1000, 64)])
def test_network_table(ctx, nt, hidden):
    p, net = seeded_net(hidden)
    net.sync(ctx)
    tab = tm.tm_wnet_table(ctx, net, nt, 16.0).cpu().numpy().astype(np.float64)
    ref = lw.table_pairs(lw.network_table(p, nt, 16.0, bf16=bf16_round))
    print(f"table nt={nt} relerr {relerr(tab[:, 0], ref[:, 0]):.2e}", flush=True)
    assert relerr(tab[:, 0], ref[:, 0]) < 2e-3
    assert np.max(np.abs(tab[:, 1] - ref[:, 1])) < 4e-3 * np.max(np.abs(ref[:, 0]))
    assert tab[-1, 1] == 0.0


def host_table(nt=256, xmax=16.0):
    xg = lw.table_grid(nt, xmax)
    v = (xg - 1.0) / (xg + 1.0) + 0.02 * np.sin(3.0 * xg)
    return lw.table_pairs(v.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("n1,n2,P,k", [(32, 32, 9, 4), (8, 8, 37, 6), (128, 64, 3, 2)])
def test_power_loss_and_table_gradient(ctx, n1, n2, P, k):
    masks, T, I64, v0 = data(n1, n2, P, 980 + n1)
    I, Iv = device_intensities(I64)
    tab = host_table()
    m = masks.astype(np.complex64).astype(np.complex128)
    # the device interpolates from (value, slope) pairs in FP32; the reference table is the same values
    vals = tab[:, 0].astype(np.float32).astype(np.float64)
    Lref, gref = lw.power_loss(ops.FFTOp(m, n1, n2), Iv, T.astype(np.complex128), v0.astype(np.complex128), vals, k)
    loss, dtab = tm.tm_wtab_power_grad(ctx, c64(masks), I, c64(T), c64(v0), n1, n2, f32(tab), k)
    loss = float(loss.item())
    dtab = dtab.cpu().numpy()
    print(f"power grad {n1}x{n2} P={P} k={k}: loss {loss:.6f} vs {Lref:.6f}, grad relerr {relerr(dtab, gref):.2e}",
          flush=True)
    assert abs(loss - Lref) < 1e-5 * max(1.0, abs(Lref))
    assert relerr(dtab, gref) < 1e-3


def test_train_step_is_the_first_adam_step_of_the_reference_gradient(ctx):
    # one training step from known weights: Adam's first step moves every parameter by
    # -lr sign(gradient); the gradient is the reference chain table gradient -> network backward
    n1, n2, P, k, nt, hidden, lr = 16, 16, 8, 3, 64, 32, 1e-3
    masks, T, I64, v0 = data(n1, n2, P, 990)
    I, Iv = device_intensities(I64)
    p, net = seeded_net(hidden, seed=12)
    net.sync(ctx)
    W0 = [w.cpu().numpy().astype(np.float64) for w in net.W]
    loss = torch.zeros((1,), dtype=torch.float32, device=dev())
    tm.tm_wnet_train_step(ctx, net, c64(masks), I, c64(T), c64(v0), n1, n2, k, nt, 16.0, lr, loss)
    vals = lw.network_table(p, nt, 16.0, bf16=bf16_round)
    m = masks.astype(np.complex64).astype(np.complex128)
    Lref, dO = lw.power_loss(ops.FFTOp(m, n1, n2), Iv, T.astype(np.complex128), v0.astype(np.complex128), vals, k)
    assert abs(float(loss.item()) - Lref) < 1e-4
    X = lw.table_features(lw.table_grid(nt))
    _, cache = omlp.forward({kk: (bf16_round(v) if kk.startswith("W") else v) for kk, v in p.items()}, bf16_round(X))
    grads = omlp.backward(p, cache, dO[:, None])
    for l, name in enumerate(("W1", "W2", "W3")):
        step = net.W[l].cpu().numpy().astype(np.float64) - W0[l]
        g = grads[name]
        big = np.abs(g) > 1e-2 * np.max(np.abs(g))
        agree = np.mean(np.sign(step[big]) == -np.sign(g[big]))
        print(f"layer {l}: {big.sum()} large gradients, sign agreement {agree:.4f}", flush=True)
        assert agree > 0.99
        assert np.allclose(np.abs(step[big]), lr, rtol=0.05)


@pytest.mark.parametrize("k", [1, 2, 3, 12])
def test_learned_lanczos_start(ctx, k):
    n1, n2, P = 32, 32, 21
    masks, T, I64, v0 = data(n1, n2, P, 995)
    I, Iv = device_intensities(I64)
    tab = host_table()
    tm.tm_set_weight_table(ctx, f32(tab), 16.0)
    tt = c64(v0)
    tm.tm_retrieve(ctx, c64(masks), I, tt, n1, n2, tm.retrieve_opts("er", iters=0, start="learned", spectral_iters=k))
    m = masks.astype(np.complex64).astype(np.complex128)
    w = lw.table_weights(tab[:, 0].astype(np.float32).astype(np.float64), lw.normalised(Iv))
    ref = rt.spectral_lanczos(ops.FFTOp(m, n1, n2), Iv, v0.astype(np.complex128), k, weights=w)
    got = tt.cpu().numpy().astype(np.complex128)
    print(f"learned lanczos k={k} relerr {relerr(got, ref):.2e} 1-fid {1 - rt.fidelity(got, ref).min():.2e}",
          flush=True)
    if k <= 3:
        assert relerr(got, ref) < 1e-5 * k
    else:
        assert 1 - rt.fidelity(got, ref).min() < 1e-4


def test_retrieve_learned_fallback(ctx):
    n1, n2, P = 32, 32, 64
    masks, T, I64, v0 = data(n1, n2, P, 996)
    I, _ = device_intensities(I64)
    tm.tm_set_weight_table(ctx, f32(host_table()), 16.0)
    mk = c64(masks)
    opts = tm.retrieve_opts("er_cyclic", iters=3, start="learned", spectral_iters=10, spectral_tau=3.0)
    # no fallback: the same as tm_retrieve from the learned start
    ta, tb = c64(v0), c64(v0)
    ra = tm.tm_retrieve(ctx, mk, I, ta, n1, n2, opts)
    rb, nf = tm.tm_retrieve_learned(ctx, mk, I, tb, n1, n2, opts, rho_fallback=1e30)
    assert nf == 0
    assert torch.equal(ta, tb) and torch.equal(ra, rb)
    # every row redone from the plain start: each keeps the result with the lower residual
    plain = tm.retrieve_opts("er_cyclic", iters=3, start="lanczos", spectral_iters=10, spectral_tau=3.0)
    tp = c64(v0)
    rp = tm.tm_retrieve(ctx, mk, I, tp, n1, n2, plain)
    tc = c64(v0)
    rc, nf = tm.tm_retrieve_learned(ctx, mk, I, tc, n1, n2, opts, rho_fallback=0.0)
    assert nf == P
    sa, sp, sc = tm.decode_stats(ra), tm.decode_stats(rp), tm.decode_stats(rc)
    take = sp.rho.numpy() < sa.rho.numpy()
    assert np.array_equal(sc.rho.numpy(), np.where(take, sp.rho.numpy(), sa.rho.numpy()))
    want = np.where(take[:, None], tp.cpu().numpy(), ta.cpu().numpy())
    assert np.array_equal(tc.cpu().numpy(), want)
