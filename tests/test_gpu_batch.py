"""Uneven batches (one persistent launch per iteration over every problem)
and the FFT digit-order autotuner."""
import json
import os

import numpy as np
import pytest
import torch

import paper_2302_13524_amd as tm
import tm_synth
from oracle import operators as ops
from oracle import retrieval as rt

from gpu_util import c64, dev, device_intensities, f32, oracle_intensities, relerr

pytestmark = pytest.mark.gpu

SHAPES = [(32, 32, 37), (64, 32, 9), (64, 64, 5), (128, 64, 3)]


@pytest.fixture(scope="module")
def ctx():
    c = tm.Context(0)
    yield c
    c.close()


def make_problems(ctx, shapes, cfg=970, bf16=True):
    out = []
    for i, (n1, n2, P) in enumerate(shapes):
        N = n1 * n2
        mh = tm_synth.mask_phases(4, N, tm_synth.rng(cfg + i, 0))
        Th = tm_synth.tm_iid(P, N, tm_synth.rng(cfg + i, 1))
        masks, T = c64(mh), c64(Th)
        I, Iv = device_intensities(oracle_intensities(mh, Th, n1, n2), bf16)
        seed = c64(tm_synth.random_start(P, N, np.ones(P), tm_synth.rng(cfg + i, 3)))
        out.append({"n1": n1, "n2": n2, "masks": masks, "I": I, "Iv": Iv, "t": seed.clone(), "seed": seed, "T": T,
                    "stats": torch.empty((P, tm.ROW_STATS_BYTES), dtype=torch.uint8, device=dev())})
    return out


def opts(mom=0.0, sp=5, iters=4, method="er", start="spectral"):
    return tm.retrieve_opts(method, iters=iters, start=start, spectral_iters=sp, bf16=True, er_momentum=mom)


def singles(ctx, probs, mom=0.0, sp=5, iters=4, method="er", start="spectral"):
    res = []
    for p in probs:
        t = p["seed"].clone()
        tm.tm_retrieve(ctx, p["masks"], p["I"], t, p["n1"], p["n2"], opts(mom, sp, iters, method, start))
        res.append(t)
    return res


@pytest.mark.parametrize("graph,mom,sp,iters,method,start", [
    (False, 0.0, 5, 4, "er", "spectral"), (True, 0.0, 5, 4, "er", "spectral"), (True, 0.8, 4, 3, "er", "spectral"),
    (True, 0.0, 4, 3, "er_cyclic", "spectral"), (False, 0.0, 3, 2, "er_cyclic", "spectral"),
    (True, 0.0, 6, 2, "er_cyclic", "lanczos"), (False, 0.0, 1, 1, "er_cyclic", "lanczos")])
def test_batch_equals_single_problem_runs(ctx, graph, mom, sp, iters, method, start):
    probs = make_problems(ctx, SHAPES)
    ref = singles(ctx, probs, mom, sp, iters, method, start)
    b = tm.Batch(ctx, probs, opts(mom, sp, iters, method, start), use_graph=graph)
    for rep in range(3):
        for p in probs:
            p["t"].copy_(p["seed"])
        b.run()
        torch.cuda.synchronize()
        for p, r in zip(probs, ref):
            assert torch.equal(p["t"], r), (rep, p["n1"], p["n2"])
        # eager work between replays
        ref = singles(ctx, probs, mom, sp, iters, method, start)
    st = tm.decode_stats(probs[0]["stats"])
    assert np.all(st.iters.numpy() == iters)
    b.close()


def test_batch_takes_the_digit_order_of_a_wider_configuration(ctx):
    # configuration 3 (eight values per thread, digit order 1) on every grid:
    # the batch runs its sixteen-value bodies in digit order 1, so it equals
    # single-problem runs in configuration 1
    probs = make_problems(ctx, SHAPES, cfg=975)
    try:
        for p in probs:
            tm.tm_set_config(ctx, p["n1"], p["n2"], 3)
        b = tm.Batch(ctx, probs, opts(0.0, 3, 2, "er_cyclic", "lanczos"), use_graph=True)
        for p in probs:
            tm.tm_set_config(ctx, p["n1"], p["n2"], 1)
        ref = singles(ctx, probs, 0.0, 3, 2, "er_cyclic", "lanczos")
        for p in probs:
            p["t"].copy_(p["seed"])
        b.run()
        torch.cuda.synchronize()
        for p, r in zip(probs, ref):
            assert torch.equal(p["t"], r), (p["n1"], p["n2"])
        b.close()
    finally:
        for p in probs:
            tm.tm_set_config(ctx, p["n1"], p["n2"], 0)


def test_batch_rows_match_oracle(ctx):
    probs = make_problems(ctx, SHAPES, cfg=980)
    o = tm.retrieve_opts("er", iters=1, start="given", bf16=True)
    b = tm.Batch(ctx, probs, o, use_graph=True)
    b.run()
    torch.cuda.synchronize()
    for p in probs:
        m = p["masks"].cpu().numpy().astype(np.complex128)
        ref = rt.er_step(ops.FFTOp(m, p["n1"], p["n2"]), p["Iv"], p["seed"].cpu().numpy().astype(np.complex128))
        assert relerr(p["t"].cpu().numpy(), ref) < 1e-5
    b.close()


def test_rejects_uncompiled_batch_grid(ctx):
    probs = make_problems(ctx, [(16, 16, 4)], cfg=990)
    with pytest.raises(tm.TMError, match="not compiled for batches"):
        tm.Batch(ctx, probs, opts())


@pytest.mark.parametrize("n1,n2", [(128, 64), (32, 32), (64, 32)])
def test_digit_order_variant_parity(ctx, n1, n2):
    P = 7
    masks, T = tm_synth.mask_phases(4, n1 * n2, tm_synth.rng(5, 0)), tm_synth.tm_iid(P, n1 * n2, tm_synth.rng(5, 1))
    I = ops.intensities(ops.FFTOp(masks.astype(np.complex64).astype(np.complex128), n1, n2),
                        T.astype(np.complex64).astype(np.complex128))
    t0 = T + 0.5 * tm_synth.tm_iid(P, n1 * n2, tm_synth.rng(5, 3))
    m = masks.astype(np.complex64).astype(np.complex128)
    ref = rt.er_step(ops.FFTOp(m, n1, n2), I.astype(np.float32).astype(np.float64), t0.astype(np.complex64).astype(np.complex128))
    for v in (0, 1):
        tm.tm_set_variant(ctx, n1, n2, v)
        tt = c64(t0)
        tm.tm_retrieve(ctx, c64(masks), f32(I), tt, n1, n2, tm.retrieve_opts("er", iters=1))
        y = tm.tm_forward(ctx, c64(masks), c64(T), n1, n2).cpu().numpy()
        assert relerr(tt.cpu().numpy(), ref) < 1e-5, v
        assert relerr(y, ops.FFTOp(m, n1, n2).forward(T.astype(np.complex64).astype(np.complex128))) < 1e-5
    tm.tm_set_variant(ctx, n1, n2, 0)


def test_autotune_times_and_caches(ctx, tmp_path):
    cache = str(tmp_path / "tune.json")
    e = tm.autotune(ctx, 128, 64, 4, 256, bf16=True, cache=cache)
    assert e["variant"] in (0, 1) and all(t > 0 for t in e["us"])
    table = json.load(open(cache))
    assert "gfx950:128x64:K4:bf16" in table
    e2 = tm.autotune(ctx, 128, 64, 4, 256, bf16=True, cache=cache)  # from the cache
    assert e2 == table["gfx950:128x64:K4:bf16"]
    tm.tm_set_variant(ctx, 128, 64, 0)
