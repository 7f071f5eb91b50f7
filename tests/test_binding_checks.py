"""Host-side argument checks of the Python binding (no GPU, no library call):
every wrapper compares the shape, dtype and device of each tensor with the
sizes it passes to the C entry point and raises TMError before anything is
launched. The context below has no library, so a wrapper that got past its
checks would fail with AttributeError instead of TMError."""
import pytest
import torch

import paper_2302_13524_amd as tm


class _NoLib:
    lib = None
    h = None


CTX = _NoLib()
K, n1, n2 = 4, 8, 8
N = n1 * n2
P = 3


def c64(*shape):
    return torch.zeros(shape, dtype=torch.complex64)


def f32(*shape):
    return torch.zeros(shape, dtype=torch.float32)


def raises(fn, *a, match=None, **kw):
    with pytest.raises(tm.TMError, match=match):
        fn(*a, **kw)


def test_forward_and_adjoint_shapes():
    raises(tm.tm_forward, CTX, c64(K, N), c64(P, N + 1), n1, n2, match="t: shape")
    raises(tm.tm_forward, CTX, c64(K, N), c64(P, N), n1, n2 * 2, match="grid")
    raises(tm.tm_forward, CTX, c64(K, N).to(torch.complex128), c64(P, N), n1, n2, match="masks: dtype")
    raises(tm.tm_forward, CTX, c64(K, N), c64(P, N), n1, n2, intensity=True, out=f32(P, K, N - 1),
           match="out: shape")
    raises(tm.tm_forward, CTX, c64(K, N), c64(P, N), n1, n2, intensity=True, bf16=True, out=f32(P, K, N),
           match="out: dtype")
    raises(tm.tm_adjoint, CTX, c64(K, N), c64(P, K + 1, N), n1, n2, match="y: shape")
    raises(tm.tm_adjoint, CTX, c64(K, N), c64(P, K, N), n1, n2, out=c64(P + 1, N), match="out: shape")
    raises(tm.tm_adjoint, CTX, c64(K, N), c64(P, N), n1, n2, match="y must be")


def test_intensity_consumers_check_I():
    for fn in (tm.tm_gradient, tm.tm_amp_gradient, tm.tm_residual_f64):
        raises(fn, CTX, c64(K, N), f32(P, K, N - 1), c64(P, N), n1, n2, match="I: shape")
        raises(fn, CTX, c64(K, N), f32(P + 1, K, N), c64(P, N), n1, n2, match="I: shape")
        raises(fn, CTX, c64(K, N), torch.zeros((P, K, N), dtype=torch.float64), c64(P, N), n1, n2,
               match="I: dtype")
        raises(fn, CTX, c64(K, N), f32(P, K, N), f32(P, N), n1, n2, match="t: dtype")
    raises(tm.tm_retrieve, CTX, c64(K, N), f32(P, K, N // 2), c64(P, N), n1, n2, match="I: shape")
    opts = tm.retrieve_opts("er", bf16=True)
    raises(tm.tm_retrieve, CTX, c64(K, N), f32(P, K, N), c64(P, N), n1, n2, opts, match="opts.I_dtype")


def test_defocus_arguments():
    nf1 = nf2 = 8
    Nd = 5
    pix = torch.zeros((P,), dtype=torch.int32)
    phi = torch.zeros((P,), dtype=torch.float64)
    Id = f32(Nd, 2 * nf1, 2 * nf2)
    raises(tm.tm_phase_objective, CTX, pix, c64(P, N), c64(Nd, N), f32(Nd, nf1, nf2), (1, .5, .2, 20), phi,
           nf1, nf2, match="I_d: shape")
    raises(tm.tm_phase_objective, CTX, pix.long(), c64(P, N), c64(Nd, N), Id, (1, .5, .2, 20), phi, nf1, nf2,
           match="pix: dtype")
    raises(tm.tm_phase_offset_correct, CTX, pix, c64(P, N), c64(Nd, N + 1), Id, (1, .5, .2, 20), phi, nf1, nf2,
           match="theta: shape")
    raises(tm.tm_phase_offset_correct, CTX, pix, c64(P, N), c64(Nd, N), Id, (1, .5, .2, 20),
           phi.float(), nf1, nf2, match="phi: dtype")
    raises(tm.tm_defocus_forward, CTX, pix[:2], c64(P, N), c64(Nd, N), (1, .5, .2, 20), phi, nf1, nf2,
           match="pix: shape")
    rec = torch.zeros((8,), dtype=torch.float64)
    raises(tm.tm_phase_offset_correct_async, CTX, pix, c64(P, N), c64(Nd, N + 1), Id, (1, .5, .2, 20), phi, nf1,
           nf2, rec, 10, match="theta: shape")
    for bad in (torch.zeros((6,), dtype=torch.float64), torch.zeros((8,), dtype=torch.float32),
                torch.zeros((8, 2), dtype=torch.float64)[:, 0]):
        raises(tm.tm_phase_offset_correct_async, CTX, pix, c64(P, N), c64(Nd, N), Id, (1, .5, .2, 20), phi, nf1,
               nf2, bad, 10, match="rec")


def test_other_entry_points():
    raises(tm.tm_dense_gradient, CTX, c64(K * N, N), f32(P, K * N - 1), c64(P, N), match="I: shape")
    raises(tm.tm_foci_power_ratio, CTX, c64(10, N), c64(2, N - 1), torch.zeros(10, dtype=torch.int32), 4, 4,
           match="tm_est: shape")
    raises(tm.tm_foci_power_ratio, CTX, c64(10, N), c64(2, N), torch.zeros(9, dtype=torch.int32), 4, 4,
           match="pix: shape")
    raises(tm.tm_propagate_tm, CTX, c64(P, N), torch.zeros(P + 1, dtype=torch.int32), 8, 8, (1, .5, .2, 1),
           match="pix: shape")
    raises(tm.tm_pre_fiber_mask, CTX, f32(16), match="energy: dtype")
    raises(tm.tm_pre_gather, CTX, torch.zeros((4, 8, 8), dtype=torch.int16), torch.zeros(3, dtype=torch.int64),
           match="pix: dtype")
    raises(tm.tm_gemm_bf16, CTX, torch.zeros((4, 8), dtype=torch.bfloat16), torch.zeros((9, 2), dtype=torch.bfloat16),
           match="B: shape")
    raises(tm.tm_gemm_bf16, CTX, f32(4, 8), torch.zeros((8, 2), dtype=torch.bfloat16), match="A: dtype")
