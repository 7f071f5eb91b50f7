"""GPU checks of the learned-start network: the MFMA GEMM tile against an
exact product, gradients against the FP64 oracle, the start rows, and a
training step that lowers the loss."""
import numpy as np
import pytest
import torch

import paper_2302_13524_amd as tm
import tm_synth
from oracle import mlp as omlp
from oracle import operators as ops

from gpu_util import c64, dev, f32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tm.Context(0)
    yield c
    c.close()


def bf16_round(x):
    return torch.as_tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()


@pytest.mark.parametrize("M,N,K", [(128, 128, 32), (200, 72, 40), (64, 300, 96), (1, 5, 3), (300, 264, 200)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_gemm_tile_matches_exact_product(ctx, M, N, K, ta, tb):
    g = torch.Generator().manual_seed(M * 7 + N + K + 3 * ta + tb)
    A = torch.randn((K, M) if ta else (M, K), generator=g).to(torch.bfloat16)
    B = torch.randn((N, K) if tb else (K, N), generator=g).to(torch.bfloat16)
    C = tm.tm_gemm_bf16(ctx, A.to(dev()), B.to(dev()), bool(ta), bool(tb)).cpu().numpy().astype(np.float64)
    a = A.to(torch.float64).numpy()
    b = B.to(torch.float64).numpy()
    ref = (a.T if ta else a) @ (b.T if tb else b)
    assert np.max(np.abs(C - ref)) <= 2e-6 * K * max(1.0, np.max(np.abs(ref)))


def small_net(N=16, K=4, H=32, seed=3):
    g = np.random.default_rng(seed)
    p = omlp.init_params(K * N, H, 2 * N, g)
    for k in ("b1", "b2", "b3"):
        p[k] = 0.05 * g.standard_normal(p[k].shape)
    for k in ("W1", "W2", "W3"):
        p[k] = bf16_round(p[k])  # the GPU multiplies BF16 copies of the weights
    net = tm.MLP(K * N, H, 2 * N, weights=[(p["W1"], p["b1"]), (p["W2"], p["b2"]), (p["W3"], p["b3"])])
    return p, net


def small_data(N=16, K=4, B=24, cfg=960):
    masks = tm_synth.mask_phases(K, N, tm_synth.rng(cfg, 0))
    T = tm_synth.tm_iid(B, N, tm_synth.rng(cfg, 1))
    I = ops.intensities(ops.FFTOp(masks, 4, N // 4), T)
    I = tm_synth.poisson_counts(I, 1e4, tm_synth.rng(cfg, 2)).astype(np.float32)
    return T.astype(np.complex64), I


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))


def test_gradients_match_oracle(ctx):
    N, K = 16, 4
    p, net = small_net()
    net.sync(ctx)
    T, I = small_data()
    dW, db, loss = tm.tm_mlp_gradients(ctx, net, f32(I), c64(T), K, N)
    X = bf16_round(omlp.features(I.astype(np.float64)))
    s = omlp.row_scale(I.astype(np.float64), K, N)
    target = T.astype(np.complex128) / s[:, None]
    o, cache = omlp.forward(p, X)
    L, dout = omlp.loss_and_dout(o, target)
    grads = omlp.backward(p, cache, dout)
    print("loss gpu", loss.mean().item(), "oracle", L)
    assert abs(loss.mean().item() - L) <= 1e-2 * abs(L)
    for l, (kw, kb) in enumerate((("W1", "b1"), ("W2", "b2"), ("W3", "b3"))):
        ew, eb = rel(dW[l].cpu().numpy(), grads[kw]), rel(db[l].cpu().numpy(), grads[kb])
        print(kw, ew, kb, eb)
        assert ew < 3e-2 and eb < 3e-2


def test_start_rows_match_oracle(ctx):
    N, K = 16, 4
    p, net = small_net(seed=5)
    net.sync(ctx)
    T, I = small_data(B=20, cfg=961)
    t0 = tm.tm_mlp_start(ctx, net, f32(I), K, N).cpu().numpy()
    X = bf16_round(omlp.features(I.astype(np.float64)))
    o, _ = omlp.forward(p, X)
    u = omlp.split_complex(o)
    ref = u / np.linalg.norm(u, axis=1, keepdims=True) * omlp.row_scale(I.astype(np.float64), K, N)[:, None]
    fid = np.abs(np.sum(np.conj(t0) * ref, 1)) ** 2 / (np.sum(np.abs(t0) ** 2, 1) * np.sum(np.abs(ref) ** 2, 1))
    assert np.all(fid > 0.999)
    assert np.allclose(np.sum(np.abs(t0) ** 2, 1), np.sum(np.abs(ref) ** 2, 1), rtol=1e-4)


def test_training_step_lowers_loss(ctx):
    # memorising a small batch: the loss must fall well below its start
    N, K = 16, 4
    _, net = small_net(seed=7, H=64)
    net.sync(ctx)
    T, I = small_data(B=32, cfg=962)
    It, Tt = f32(I), c64(T)
    loss = torch.empty(32, dtype=torch.float32, device=dev())
    tm.tm_mlp_train_step(ctx, net, It, Tt, K, N, 3e-3, loss)
    first = loss.mean().item()
    for _ in range(300):
        tm.tm_mlp_train_step(ctx, net, It, Tt, K, N, 3e-3, loss)
    last = loss.mean().item()
    print("loss", first, "->", last)
    assert last < 0.5 * first
