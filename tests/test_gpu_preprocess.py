"""GPU parity of the preprocessing entry points (half-sampling, fiber mask,
per-pixel rows) against the oracle: bit-exact for uint16 stacks, where every
sum is an exact integer in FP64."""
import json
import os

import numpy as np
import pytest
import torch

import paper_2302_13524_amd as tm
import tm_synth
from oracle import operators as ops
from oracle import preprocess as pp
from oracle import retrieval as rt

from gpu_util import c64, dev, f32

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "preprocess_example.json")


@pytest.fixture(scope="module")
def ctx():
    c = tm.Context(0)
    yield c
    c.close()


def u16(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint16)).to(dev())


def test_hand_example(ctx):
    d = json.load(open(GOLD))
    st = u16(np.array(d["stack"]))
    E = tm.tm_pre_energy(ctx, st)
    assert E.cpu().numpy().tolist() == d["energy"]
    for frac in ("0.999", "0.7", "0.4"):
        assert tm.tm_pre_fiber_mask(ctx, E, float(frac)).cpu().numpy().tolist() == d["mask_" + frac]
    pix = torch.tensor(d["mask_0.7"], dtype=torch.int32, device=dev())
    assert tm.tm_pre_gather(ctx, st, pix).cpu().numpy().tolist() == d["rows_0.7"]


@pytest.mark.parametrize("n,H,W,radius", [(37, 6, 10, 2.0), (200, 32, 32, 10.0), (1000, 128, 128, 54.0),
                                          (70, 2, 2, 1.0), (65, 256, 128, 40.0)])
def test_uint16_stacks_bit_exact(ctx, n, H, W, radius):
    print(f"preprocess n={n} H={H} W={W}", flush=True)
    g = tm_synth.rng(960 + H, 0)
    stack = tm_synth.camera_stack(n, H, W, radius, g)
    st = u16(stack)
    E = tm.tm_pre_energy(ctx, st).cpu().numpy()
    Eo = pp.energy(stack)
    assert np.array_equal(E, Eo)
    for frac in (0.999, 0.5, 1.0):
        pix = tm.tm_pre_fiber_mask(ctx, torch.from_numpy(Eo).to(dev()), frac)
        po = pp.fiber_mask(Eo, frac)
        assert np.array_equal(pix.cpu().numpy(), po), frac
    rows = tm.tm_pre_gather(ctx, st, pix)
    ro = pp.gather_rows(stack, po).astype(np.float32)
    assert np.array_equal(rows.cpu().numpy(), ro)
    rb = tm.tm_pre_gather(ctx, st, pix, bf16=True)
    assert torch.equal(rb.cpu(), torch.from_numpy(ro).to(torch.bfloat16))


def test_float_stack(ctx):
    # float32 images: energies agree to rounding; the mask of the oracle's
    # energies, computed on the device, equals the oracle's mask of them, and
    # the rows gathered for it equal the oracle's
    g = tm_synth.rng(970, 0)
    stack = (tm_synth.camera_stack(300, 64, 64, 25.0, g).astype(np.float32) * 0.37).astype(np.float32)
    st = f32(stack)
    E = tm.tm_pre_energy(ctx, st)
    Eo = pp.energy(stack)
    assert np.max(np.abs(E.cpu().numpy() - Eo)) <= 1e-12 * np.max(Eo)
    po = pp.fiber_mask(Eo, 0.999)
    pix = tm.tm_pre_fiber_mask(ctx, torch.from_numpy(Eo).to(dev()), 0.999)
    assert np.array_equal(pix.cpu().numpy(), po)
    assert np.array_equal(tm.tm_pre_gather(ctx, st, pix).cpu().numpy(), pp.gather_rows(stack, po))


def test_fiber_disk_is_the_mask(ctx):
    # the mask lies inside the fiber core; the 0.1 % of energy it leaves out
    # drops at most a few of the dimmest core pixels (speckle varies per pixel)
    stack = tm_synth.camera_stack(256, 128, 128, 54.0, tm_synth.rng(971, 0))
    E = tm.tm_pre_energy(ctx, u16(stack))
    pix = tm.tm_pre_fiber_mask(ctx, E, 0.999).cpu().numpy()
    assert np.array_equal(pix, pp.fiber_mask(pp.energy(stack), 0.999))
    disk = np.flatnonzero(tm_synth.fiber_disk(128, 128, 54.0)[0::2, 0::2].reshape(-1))
    assert np.all(np.isin(pix, disk)) and len(pix) >= 0.995 * len(disk)


def test_edge_cases_and_errors(ctx):
    z = u16(np.zeros((5, 8, 8)))
    assert tm.tm_pre_fiber_mask(ctx, tm.tm_pre_energy(ctx, z), 0.999).numel() == 0
    empty = torch.empty((0,), dtype=torch.int32, device=dev())
    assert tm.tm_pre_gather(ctx, z, empty).shape == (0, 5)
    with pytest.raises(tm.TMError, match="even sizes"):
        tm.tm_pre_energy(ctx, u16(np.zeros((2, 7, 8))))
    with pytest.raises(tm.TMError, match="npix"):
        tm.tm_pre_fiber_mask(ctx, torch.ones(8193, dtype=torch.float64, device=dev()), 0.999)
    with pytest.raises(tm.TMError, match="frac"):
        tm.tm_pre_fiber_mask(ctx, torch.ones(16, dtype=torch.float64, device=dev()), 0.0)
    with pytest.raises(tm.TMError, match="outside the half-sampled grid"):
        tm.tm_pre_gather(ctx, z, torch.tensor([0, 16], dtype=torch.int32, device=dev()))


def test_camera_layout_to_retrieval(ctx):
    # full-resolution camera: every camera pixel has its own TM row; the rows
    # of the pixels inside the fiber are speckle, outside they are dim. The
    # preprocessing picks the fiber pixels of the half-sampled grid and their
    # rows, which tm_retrieve then recovers (noiseless, K = 4, 8 x 8 modes).
    n1 = n2 = 8
    N, K, H = n1 * n2, 4, 16
    masks = tm_synth.mask_phases(K, N, tm_synth.rng(972, 0))
    inside = tm_synth.fiber_disk(H, H, 6.0).reshape(-1)
    T = tm_synth.tm_iid(H * H, N, tm_synth.rng(972, 1)) * np.where(inside, 1.0, 1e-3)[:, None]
    I = ops.intensities(ops.FFTOp(masks, n1, n2), T).reshape(H * H, K * N)  # [camera pixel][image]
    stack = I.T.reshape(K * N, H, H).astype(np.float32)
    st = f32(stack)
    pix = tm.tm_pre_fiber_mask(ctx, tm.tm_pre_energy(ctx, st), 0.999)
    half = tm_synth.fiber_disk(H, H, 6.0)[0::2, 0::2].reshape(-1)
    assert np.array_equal(pix.cpu().numpy(), np.flatnonzero(half))
    rows = tm.tm_pre_gather(ctx, st, pix).contiguous()
    P = rows.shape[0]
    cam = np.flatnonzero(half)  # half-grid index q -> camera pixel (2y, 2x)
    cam = (2 * (cam // (H // 2))) * H + 2 * (cam % (H // 2))
    v0 = c64(tm_synth.random_start(P, N, np.ones(P), tm_synth.rng(972, 3)))
    tm.tm_retrieve(ctx, c64(masks), rows.view(P, K, N), v0, n1, n2,  # [pixel][image] is [P][K][N]
                   tm.retrieve_opts("er", iters=150, start="spectral", spectral_iters=40, spectral_lower=0.0))
    fid = rt.fidelity(v0.cpu().numpy().astype(np.complex128), T[cam])
    assert fid.mean() > 0.99
