"""GPU parity of the complex FP32 matrix-core GEMM (tm_cgemm_f32) against
the exact product of the same FP32 inputs (numpy, complex128)."""
import numpy as np
import pytest
import torch

import paper_2302_13524_amd as tm

from gpu_util import dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tm.Context(0)
    yield c
    c.close()


def _rand(shape, g):
    return (g.standard_normal(shape) + 1j * g.standard_normal(shape)).astype(np.complex64)


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (37, 53, 19), (128, 128, 8), (200, 300, 100), (257, 129, 1000),
                                   (64, 520, 33)])
@pytest.mark.parametrize("trans_b", [False, True])
@pytest.mark.parametrize("conj_c", [False, True])
def test_cgemm_matches_exact_product(ctx, M, N, K, trans_b, conj_c):
    # ragged tiles (128 x 128 x 8), odd leading dimensions (scalar loads), one
    # and several K steps; the error bound: FP32 products summed over K
    g = np.random.default_rng(M * 7 + N * 3 + K)
    A = _rand((M, K), g)
    B = _rand((N, K) if trans_b else (K, N), g)
    C = tm.tm_cgemm_f32(ctx, torch.from_numpy(A).to(dev()), torch.from_numpy(B).to(dev()), trans_b, conj_c)
    ref = A.astype(np.complex128) @ (B.T if trans_b else B).astype(np.complex128)
    if conj_c:
        ref = np.conj(ref)
    got = C.cpu().numpy().astype(np.complex128)
    scale = np.sqrt(K) * 2.0  # typical |C| for unit complex normals
    err = np.max(np.abs(got - ref)) / scale
    print(f"cgemm {M}x{N}x{K} trans_b={trans_b} conj={conj_c}: max err / sqrt(K) {err:.3e}")
    assert err < 1e-5 * max(1.0, np.log2(K))


def test_cgemm_rejects_bad_arguments(ctx):
    A = torch.zeros((4, 3), dtype=torch.complex64, device=dev())
    with pytest.raises(tm.TMError):
        tm.tm_cgemm_f32(ctx, A, torch.zeros((5, 4), dtype=torch.complex64, device=dev()))
    with pytest.raises(tm.TMError):
        tm.tm_cgemm_f32(ctx, A.to(torch.complex128), torch.zeros((3, 4), dtype=torch.complex64, device=dev()))
    # M or N zero: nothing to do
    C = tm.tm_cgemm_f32(ctx, torch.zeros((0, 3), dtype=torch.complex64, device=dev()),
                        torch.zeros((3, 4), dtype=torch.complex64, device=dev()))
    assert C.shape == (0, 4)
