"""Pins of the FP64 learned-start network oracle: backward pass against
central finite differences, loss invariances, Adam's first step. CPU only."""
import numpy as np

from oracle import mlp


def tiny(seed=0, n_in=12, H=7, N=4, B=5):
    g = np.random.default_rng(seed)
    p = mlp.init_params(n_in, H, 2 * N, g)
    for k in ("b1", "b2", "b3"):
        p[k] = 0.1 * g.standard_normal(p[k].shape)
    X = g.random((B, n_in)) * 2
    T = g.standard_normal((B, N)) + 1j * g.standard_normal((B, N))
    return p, X, T


def total_loss(p, X, T):
    o, _ = mlp.forward(p, X)
    return mlp.loss_and_dout(o, T)[0]


def test_backward_matches_central_differences():
    p, X, T = tiny()
    o, cache = mlp.forward(p, X)
    _, dout = mlp.loss_and_dout(o, T)
    grads = mlp.backward(p, cache, dout)
    h = 1e-6
    for k in p:
        num = np.zeros_like(p[k])
        it = np.nditer(p[k], flags=["multi_index"])
        for _ in it:
            i = it.multi_index
            old = p[k][i]
            p[k][i] = old + h
            fp = total_loss(p, X, T)
            p[k][i] = old - h
            fm = total_loss(p, X, T)
            p[k][i] = old
            num[i] = (fp - fm) / (2 * h)
        assert np.max(np.abs(num - grads[k])) < 1e-6 * max(1.0, np.max(np.abs(num))), k


def test_loss_is_phase_invariant_and_zero_at_target():
    p, X, T = tiny(1)
    o, _ = mlp.forward(p, X)
    L1, _ = mlp.loss_and_dout(o, T)
    L2, _ = mlp.loss_and_dout(o, T * np.exp(1j * 0.77))
    assert abs(L1 - L2) < 1e-12
    N = T.shape[1]
    o_exact = np.concatenate([T.real, T.imag], axis=1) * np.exp(0)  # u = u*
    L0, d0 = mlp.loss_and_dout(o_exact, T * np.exp(1j * 1.3))
    assert abs(L0) < 1e-12 and np.max(np.abs(d0)) < 1e-12


def test_gelu_is_erf_form():
    x = np.array([-3.0, -0.5, 0.0, 0.5, 2.0])
    ref = np.array([-0.0040496, -0.1542688, 0.0, 0.3457312, 1.9544997])
    assert np.allclose(mlp.gelu(x), ref, atol=1e-6)
    h = 1e-6
    assert np.allclose(mlp.gelu_grad(x), (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h), atol=1e-8)


def test_adam_first_step_is_signed_learning_rate():
    # at step 1 the bias-corrected ratio m/sqrt(v) equals g/|g|
    p = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -4.0, 1e-3])}
    st = {}
    mlp.adam_step(p, g, st, lr=0.01)
    assert np.allclose(p["w"], [1.0 - 0.01, -2.0 + 0.01, 0.5 - 0.01], atol=1e-6)


def test_predicted_start_has_parseval_norm():
    p, _, _ = tiny(2, n_in=16, N=4)
    g = np.random.default_rng(3)
    I = g.random((3, 4, 4))
    t0 = mlp.predict_start(p, I, 4, 4)
    assert np.allclose(np.sum(np.abs(t0) ** 2, 1), I.reshape(3, -1).sum(1) / 16)
