"""The allocation-free entry point tm_retrieve_noalloc (C ABI) against
tm_retrieve on the same inputs: the same kernels run in the same order, so
rows and per-row records must be identical; two calls in a row, the second
with fewer rows (the shared scratch keeps the first call's values), and the
host-side rejections."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2302_13524_amd as tm
import tm_synth
from oracle import operators as ops
from oracle import retrieval as rt

from gpu_util import c64, device_intensities, problem, relerr, rounded

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tm.Context(0)
    yield c
    c.close()


def _both(ctx, masks, I, t0, n1, n2, opts):
    P = t0.shape[0]
    ta, tb = c64(t0), c64(t0)
    sa = torch.zeros((P, tm.ROW_STATS_BYTES), dtype=torch.uint8, device=ta.device)
    sb = torch.full((P, tm.ROW_STATS_BYTES), 7, dtype=torch.uint8, device=ta.device)
    rc = ctx.lib.tm_retrieve(ctx.h, tm.tm_dims(n1, n2, 4, P), masks.data_ptr(), I.data_ptr(), ta.data_ptr(),
                             ctypes.byref(opts), sa.data_ptr(), None)
    assert rc == tm.TM_OK, ctx.lib.tm_last_error(ctx.h)
    rc = ctx.lib.tm_retrieve_noalloc(ctx.h, tm.tm_dims(n1, n2, 4, P), masks.data_ptr(), I.data_ptr(),
                                     tb.data_ptr(), ctypes.byref(opts), sb.data_ptr(), None)
    assert rc == tm.TM_OK, ctx.lib.tm_last_error(ctx.h)
    torch.cuda.synchronize()
    return ta.cpu().numpy(), tb.cpu().numpy(), sa.cpu().numpy(), sb.cpu().numpy()


@pytest.mark.parametrize("method,start,bf16", [("er_cyclic", "given", False), ("er", "backprop", True)])
def test_noalloc_matches_tm_retrieve_twice(ctx, method, start, bf16):
    n1, n2 = 32, 32
    for call, (P, cfg) in enumerate(((300, 941), (77, 942))):  # second call: fewer rows, other data
        print(f"noalloc {method}/{start} bf16={bf16} call {call} P={P}", flush=True)
        masks, T, I64, _ = problem(n1, n2, 4, P, cfg=cfg, noise=1e4)
        t0 = T + 0.4 * tm_synth.tm_iid(P, n1 * n2, tm_synth.rng(cfg, 3))
        I, Iv = device_intensities(I64, bf16)
        opts = tm.retrieve_opts(method, iters=3, start=start, bf16=bf16)
        a, b, sa, sb = _both(ctx, c64(masks), I, t0, n1, n2, opts)
        assert np.array_equal(a, b)
        assert np.array_equal(sa, sb)
        # and the oracle's same steps (the existing entry point's bar)
        m, t, _ = rounded(masks, t0, I64)
        op = ops.FFTOp(m, n1, n2)
        if method == "er_cyclic":
            ref = rt.er_cyclic(m, n1, n2, Iv, t, 3)
        else:
            ref = rt.backprop_start(op, Iv)
            for _ in range(3):
                ref = rt.er_step(op, Iv, ref)
        assert relerr(b, ref) < 3e-5
        st = tm.decode_stats(torch.from_numpy(sb))
        assert np.all(st.iters.numpy() == 3)
        rho = rt.acceptance_residual(op, Iv, b.astype(np.complex128))
        assert relerr(st.rho.numpy(), rho) < 1e-6


def test_noalloc_rejections(ctx):
    lib = ctx.lib
    opts = tm.retrieve_opts("er_cyclic", iters=1)
    big = tm.tm_dims(32, 32, 4, tm.TM_NOALLOC_MAX_ROWS + 1)
    assert lib.tm_retrieve_noalloc(ctx.h, big, None, None, None, ctypes.byref(opts), None, None) == tm.TM_EINVAL
    assert b"exceeds" in lib.tm_last_error(ctx.h)
    d = tm.tm_dims(32, 32, 4, 4)
    for o in (tm.retrieve_opts("lbfgs", iters=1), tm.retrieve_opts("er_cyclic", iters=1, start="lanczos"),
              tm.retrieve_opts("er", iters=1, er_momentum=0.5)):
        assert lib.tm_retrieve_noalloc(ctx.h, d, None, None, None, ctypes.byref(o), None, None) == tm.TM_EUNSUPPORTED
    assert lib.tm_retrieve_noalloc(None, d, None, None, None, ctypes.byref(opts), None, None) == tm.TM_EINVAL
