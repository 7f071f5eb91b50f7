"""GPU parity of the TM propagated to a defocus distance against the oracle."""
import numpy as np
import pytest
import torch

import paper_2302_13524_amd as tm
import tm_synth
from oracle import foci

from gpu_util import c64, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tm.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("g1,g2,P,N,z", [(32, 32, 700, 256, 15.0), (16, 16, 150, 33, -4.0), (64, 32, 1500, 64, 40.0),
                                         (64, 64, 2286, 100, 0.0), (8, 8, 64, 7, 3.0)])
def test_propagated_tm_matches_oracle(ctx, g1, g2, P, N, z):
    print(f"propagate {g1}x{g2} P={P} N={N} z={z}", flush=True)
    if g1 == g2:
        pix = tm_synth.nearest_pixels(g1, P)
    else:
        pix = np.sort(tm_synth.rng(998, 3).choice(g1 * g2, size=P, replace=False))
    T = tm_synth.tm_iid(P, N, tm_synth.rng(998, 1))
    lam, ps, NA = 1.0, 0.5, 0.45
    out = tm.tm_propagate_tm(ctx, c64(T), torch.from_numpy(pix.astype(np.int32)).to(dev()), g1, g2,
                             (lam, ps, NA, z)).cpu().numpy()
    ref = foci.propagate_tm(T.astype(np.complex64).astype(np.complex128), pix, g1, g2, lam, ps, NA, z)
    assert out.shape == ref.shape == (g1 * g2, N)
    # FP32 2-D FFTs over g1 g2 points: error relative to the column's RMS
    rms = np.sqrt(np.mean(np.abs(ref) ** 2, axis=0))
    err = np.max(np.abs(out - ref) / np.maximum(rms, 1e-30)[None, :])
    assert err < 5e-6 * np.log2(g1 * g2)


def test_full_pupil_at_zero_distance_is_identity(ctx):
    # NA covers every frequency of the grid and z = 0: h = 1, the TM is only scattered onto the grid
    g, P, N = 32, 400, 48
    pix = tm_synth.nearest_pixels(g, P)
    T = tm_synth.tm_iid(P, N, tm_synth.rng(999, 1))
    out = tm.tm_propagate_tm(ctx, c64(T), torch.from_numpy(pix.astype(np.int32)).to(dev()), g, g,
                             (1.0, 1.0, 2.0, 0.0)).cpu().numpy()
    want = np.zeros((g * g, N), dtype=np.complex128)
    want[pix] = T
    assert np.max(np.abs(out - want)) < 1e-5


def test_errors(ctx):
    T = c64(np.ones((3, 4)))
    opt = (1.0, 0.5, 0.4, 1.0)
    with pytest.raises(tm.TMError, match="repeats"):
        tm.tm_propagate_tm(ctx, T, torch.tensor([0, 1, 1], dtype=torch.int32, device=dev()), 8, 8, opt)
    with pytest.raises(tm.TMError, match="outside the grid"):
        tm.tm_propagate_tm(ctx, T, torch.tensor([0, 1, 64], dtype=torch.int32, device=dev()), 8, 8, opt)
    with pytest.raises(tm.TMError):
        tm.tm_propagate_tm(ctx, T, torch.tensor([0, 1, 2], dtype=torch.int32, device=dev()), 12, 12, opt)
    with pytest.raises(tm.TMError, match="optics"):
        tm.tm_propagate_tm(ctx, T, torch.tensor([0, 1, 2], dtype=torch.int32, device=dev()), 8, 8, (1.0, 0.5, 0.0, 1.0))
