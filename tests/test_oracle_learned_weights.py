"""Pins of the learned spectral weighting's FP64 reference (CPU): the table
interpolation, the power-iteration training loss and its gradient, and the
weighted Lanczos start."""
import numpy as np

import tm_synth
from oracle import learned_weights as lw
from oracle import operators as ops
from oracle import retrieval as rt


def _tiny(cfg=5, P=3, n1=4, n2=4, K=4, photons=100):
    N = n1 * n2
    masks = tm_synth.mask_phases(K, N, tm_synth.rng(cfg, 0))
    T = tm_synth.tm_iid(P, N, tm_synth.rng(cfg, 1))
    op = ops.FFTOp(masks, n1, n2)
    I = tm_synth.poisson_counts(ops.intensities(op, T), photons, tm_synth.rng(cfg, 2))
    v0 = tm_synth.tm_iid(P, N, tm_synth.rng(cfg, 3))
    return op, I, T, v0


def test_table_interpolation_closed_forms():
    nt, xmax = 9, 8.0
    tab = np.array([3.0, -1.0, 2.0, 0.5, 0.0, 4.0, 4.0, -2.0, 1.0])
    xg = lw.table_grid(nt, xmax)
    assert np.array_equal(xg, np.arange(9.0))
    # exact at the grid points, linear between them, clamped outside [0, xmax]
    assert np.allclose(lw.table_weights(tab, xg, xmax), tab)
    assert np.isclose(lw.table_weights(tab, np.array([0.25]), xmax)[0], 0.75 * 3.0 + 0.25 * -1.0)
    assert np.isclose(lw.table_weights(tab, np.array([6.5]), xmax)[0], 0.5 * 4.0 + 0.5 * -2.0)
    assert np.allclose(lw.table_weights(tab, np.array([-3.0, 8.0, 100.0]), xmax), [3.0, 1.0, 1.0])
    # a linear table reproduces the line
    lin = 2.0 * xg - 1.0
    x = np.random.default_rng(0).uniform(0, 8, 50)
    assert np.allclose(lw.table_weights(lin, x, xmax), 2.0 * x - 1.0)
    # the adjoint: sum_b dtab_b T_b = sum_i g_i w_i for any table
    g = np.random.default_rng(1).standard_normal(50)
    assert np.isclose(lw.scatter_to_table(g, x, nt, xmax) @ tab, g @ lw.table_weights(tab, x, xmax))
    # the library's (value, slope) layout
    pr = lw.table_pairs(tab)
    assert np.allclose(pr[:, 0] + pr[:, 1], np.append(tab[1:], tab[-1]))


def test_power_loss_gradient_by_central_differences():
    op, I, T, v0 = _tiny()
    nt = 9
    tab = np.minimum(lw.table_grid(nt, 8.0), 3.0) + 0.1 * np.random.default_rng(1).standard_normal(nt)
    for k in (1, 4):
        L, g = lw.power_loss(op, I, T, v0, tab, k, xmax=8.0)
        fd = np.zeros(nt)
        e = 1e-6
        for b in range(nt):
            tp, tq = tab.copy(), tab.copy()
            tp[b] += e
            tq[b] -= e
            fd[b] = (lw.power_loss(op, I, T, v0, tp, k, 8.0, False)[0] - lw.power_loss(op, I, T, v0, tq, k, 8.0,
                                                                                        False)[0]) / (2 * e)
        assert np.max(np.abs(g - fd)) <= 1e-6 * max(1.0, np.max(np.abs(fd)))
        assert np.any(np.abs(fd) > 1e-4)


def test_power_loss_special_cases():
    op, I, T, v0 = _tiny()
    # constant weights: M = c K N I maps every vector to a multiple of itself, so
    # the loss is minus the seeds' own fidelity, at any step count
    for k in (1, 3):
        L, g = lw.power_loss(op, I, T, v0, np.full(5, 2.5), k, xmax=8.0)
        assert np.isclose(L, -np.mean(rt.fidelity(v0, T)))
    # k steps equal k plain power steps on A^H diag(w) A (a dense eigen-solve agrees in the limit)
    x = lw.normalised(I)
    tab = np.minimum(lw.table_grid(17, 8.0), 3.0)
    w = lw.table_weights(tab, x, 8.0)
    A = ops.DenseOp(op.masks, op.n1, op.n2).A
    u = v0 / np.linalg.norm(v0, axis=1, keepdims=True)
    for _ in range(400):
        u = np.stack([(A.conj().T * w[p].ravel()) @ (A @ u[p]) for p in range(u.shape[0])])
        u /= np.linalg.norm(u, axis=1, keepdims=True)
    top = []
    for p in range(u.shape[0]):
        M = (A.conj().T * w[p].ravel()) @ A
        ev, vec = np.linalg.eigh(M)
        top.append(vec[:, -1])
    top = np.array(top)
    L, _ = lw.power_loss(op, I, T, v0, tab, 400, xmax=8.0, grad=False)
    assert np.isclose(L, -np.mean(rt.fidelity(top, T)), atol=1e-6)


def test_weighted_lanczos_is_the_plain_start_with_its_own_weights():
    op, I, T, v0 = _tiny(P=4, n1=8, n2=8)
    w = rt.spectral_weights(I, 3.0)
    a = rt.spectral_lanczos(op, I, v0, 6, tau=3.0)
    b = rt.spectral_lanczos(op, I, v0, 6, weights=w)
    assert np.allclose(a, b)
    # a table that reproduces min(x, 3) on its grid gives the same start
    tab = np.minimum(lw.table_grid(129, 16.0), 3.0)  # x = 3 is a grid point: exact
    c = rt.spectral_lanczos(op, I, v0, 6, weights=lw.table_weights(tab, lw.normalised(I), 16.0))
    assert np.allclose(a, c)


def test_features_and_network_table_shapes():
    xg = lw.table_grid(33)
    X = lw.table_features(xg)
    assert X.shape == (33, lw.N_FEAT)
    assert np.allclose(X[:, 14], 1.0)
    assert np.allclose(X[0, :16], [0, 0, 0, 0, 1, 1, 1, 0, np.tanh(-1), np.tanh(-1.5), 0, 0, 0, 0, 1, 1])
    from oracle import mlp
    p = mlp.init_params(lw.N_FEAT, 8, 1, np.random.default_rng(0))
    v = lw.network_table(p, 33)
    o, _ = mlp.forward(p, X)
    assert np.allclose(v, o[:, 0])
