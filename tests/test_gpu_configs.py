"""GPU parity of every compiled launch configuration (digit order, values per
thread, rows per workgroup) of the Lanczos and cyclic ER steps against the
FP64 oracle, and the wide autotuner."""
import numpy as np
import pytest

import paper_2302_13524_amd as tm
import tm_synth
from oracle import operators as ops
from oracle import retrieval as rt

from gpu_util import c64, f32, problem, relerr, rounded

pytestmark = pytest.mark.gpu

OPTOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = tm.Context(0)
    yield c
    c.close()


def _fid(a, b):
    c = np.abs(np.sum(np.conj(a) * b, axis=1)) ** 2
    return c / (np.sum(np.abs(a) ** 2, axis=1) * np.sum(np.abs(b) ** 2, axis=1))


def _cases():
    try:
        tm.load()
    except tm.TMError:  # library not built: collected only
        return []
    out = []
    for n1, n2, P in [(32, 32, 21), (64, 32, 9), (64, 64, 7), (128, 64, 5)]:
        for cfg in range(8):
            if tm.tm_config_info(n1, n2, cfg) is not None:
                out.append((n1, n2, P, cfg))
    return out


@pytest.mark.parametrize("n1,n2,P,cfg", _cases())
def test_config_lanczos_and_cyclic_er(ctx, n1, n2, P, cfg):
    # in configuration cfg: three Lanczos steps of the start (per-step
    # tolerance), and two cyclic sweeps from a given start (K projections per
    # sweep, each a transform pair held to OPTOL); the context's default
    # configuration is restored afterwards
    print(f"config {cfg} grid {n1}x{n2} P={P} shape {tm.tm_config_info(n1, n2, cfg)}", flush=True)
    masks, T, I, _ = problem(n1, n2, 4, P, cfg=941, noise=1e4)
    v0 = tm_synth.random_start(P, n1 * n2, np.ones(P), tm_synth.rng(941, 3))
    t0 = T + 0.7 * tm_synth.tm_iid(P, n1 * n2, tm_synth.rng(941, 4))
    m, v, Ir = rounded(masks, v0, I)
    _, t, _ = rounded(masks, t0, I)
    k, sweeps = 3, 2
    ref_lz = rt.spectral_lanczos(ops.FFTOp(m, n1, n2), Ir, v, k, tau=2.5)
    ref_er = rt.er_cyclic(m, n1, n2, Ir, t, sweeps)
    tm.tm_set_config(ctx, n1, n2, cfg)
    try:
        tl = c64(v0)
        tm.tm_retrieve(ctx, c64(masks), f32(I), tl, n1, n2,
                       tm.retrieve_opts("er", iters=0, start="lanczos", spectral_iters=k, spectral_tau=2.5))
        assert relerr(tl.cpu().numpy().astype(np.complex128), ref_lz) < OPTOL * k
        tt = c64(t0)
        tm.tm_retrieve(ctx, c64(masks), f32(I), tt, n1, n2, tm.retrieve_opts("er_cyclic", iters=sweeps))
        assert relerr(tt.cpu().numpy().astype(np.complex128), ref_er) < OPTOL * 4 * sweeps
    finally:
        tm.tm_set_config(ctx, n1, n2, 0)


@pytest.mark.parametrize("n1,n2,P,cfg", _cases())
def test_config_lbfgs(ctx, n1, n2, P, cfg):
    # Alg. 1 and its amplitude-cost form in configuration cfg (the gradient
    # kernels and the amplitude line search in that launch shape): three
    # iterations against the oracle, as in the default configuration
    masks, T, I, _ = problem(n1, n2, 4, P, cfg=942, noise=1e4)
    t0 = T + 0.3 * tm_synth.tm_iid(P, n1 * n2, tm_synth.rng(942, 3))
    m, t, Ir = rounded(masks, t0, I)
    op = ops.FFTOp(m, n1, n2)
    iters = 3
    ref_i, _ = rt.lbfgs(op, Ir, t, iters, m=5)
    ref_a, _ = rt.lbfgs_amplitude(op, Ir, t, iters, m=5)
    tm.tm_set_config(ctx, n1, n2, cfg)
    try:
        for method, ref in (("lbfgs", ref_i), ("lbfgs_amp", ref_a)):
            tt = c64(t0)
            tm.tm_retrieve(ctx, c64(masks), f32(I), tt, n1, n2, tm.retrieve_opts(method, iters=iters, lbfgs_m=5))
            err = relerr(tt.cpu().numpy().astype(np.complex128), ref)
            print(f"config {cfg} grid {n1}x{n2} {method} relerr {err:.3e}", flush=True)
            assert err < (1e-4 * iters if method == "lbfgs" else 1e-3), (method, err)
    finally:
        tm.tm_set_config(ctx, n1, n2, 0)


def test_config_rejections(ctx):
    with pytest.raises(tm.TMError, match="not compiled"):
        tm.tm_set_config(ctx, 128, 64, 4)
    with pytest.raises(tm.TMError, match="not compiled"):
        tm.tm_set_config(ctx, 8, 8, 2)
    with pytest.raises(tm.TMError):
        tm.tm_tune_config(ctx, 128, 64, 4, 16, 5)


def test_wide_autotune_applies_a_compiled_configuration(ctx, tmp_path):
    cache = str(tmp_path / "tune.json")
    e = tm.autotune(ctx, 64, 32, 4, 900, cache=cache, space="full", reps=2)
    assert set(e["candidates"]) == {str(c) for c in range(8) if tm.tm_config_info(64, 32, c)}
    best = min(e["candidates"].values(), key=lambda c: c["lanczos_us"] + c["er_cyclic_us"])
    assert e["candidates"][str(e["config"])] == best
    # cached: applied again without timing, same entry
    e2 = tm.autotune(ctx, 64, 32, 4, 900, cache=cache, space="full")
    assert e2 == e
    tm.tm_set_config(ctx, 64, 32, 0)
