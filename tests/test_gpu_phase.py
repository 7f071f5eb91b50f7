"""GPU parity of the FP64 phase-offset correction (Sec. 2.3) against the oracle."""
import numpy as np
import pytest
import torch

import paper_2302_13524_amd as tm
import tm_synth
from oracle import defocus as df

from gpu_util import c64, dev, f32, relerr

pytestmark = pytest.mark.gpu
LAM = 1.0
PS = 0.5


@pytest.fixture(scope="module")
def ctx():
    c = tm.Context(0)
    yield c
    c.close()


def build(nf, P, N, Nd, NA, pupil_frac, cfg, noise=None):
    pix = tm_synth.nearest_pixels(nf, P)
    tm_true = tm_synth.speckle_tm(N, nf, pupil_frac, pix, tm_synth.rng(cfg, 1))
    phi_true = tm_synth.offsets(P, tm_synth.rng(cfg, 5))
    tm_est = (np.exp(-1j * phi_true)[:, None] * tm_true).astype(np.complex64)
    theta = tm_synth.defocus_phases(Nd, N, tm_synth.rng(cfg, 4)).astype(np.complex64)
    mdl = df.DefocusModel(tm_est.astype(np.complex128), theta.astype(np.complex128), pix, nf, nf, LAM, PS, NA,
                          20 * LAM)
    Id = mdl.images(phi_true)
    if noise:
        Id = tm_synth.poisson_counts(Id, noise, tm_synth.rng(cfg, 6))
    Id = Id.astype(np.float32)
    return pix, tm_est, theta, Id, phi_true, mdl


@pytest.fixture
def band(ctx, request):
    tm.tm_phase_set_band(ctx, request.param)
    yield request.param
    tm.tm_phase_set_band(ctx, True)


# NA 0.3: pupil boxes of 5, 9 and 19 bins (the last above the band limit, so
# the band setting falls back to full FFTs); NA 0.22 at 64 x 64 is the
# 15-bin box of the paper-scale workload; 70 images over an odd N take the
# c_n product's second image tile and its element-wise loads
@pytest.mark.parametrize("band", [True, False], indirect=True)
@pytest.mark.parametrize("nf,P,N,Nd,NA", [(16, 40, 24, 12, 0.3), (32, 512, 1024, 50, 0.3), (64, 2286, 8192, 50, 0.3),
                                          (64, 2286, 1024, 50, 0.22), (16, 70, 25, 70, 0.3)])
def test_objective_and_gradient(ctx, band, nf, P, N, Nd, NA):
    print(f"phase objective nf={nf} P={P} N={N} Nd={Nd} NA={NA} band={band}", flush=True)
    pix, tm_est, theta, Id, phi_true, mdl = build(nf, P, N, Nd, NA, NA, cfg=950, noise=1e4)
    phi = np.random.default_rng(1).random(P) * 2 * np.pi
    gref, grad_ref = mdl.objective(Id.astype(np.float64), phi)
    g, grad = tm.tm_phase_objective(ctx, torch.from_numpy(pix.astype(np.int32)).to(dev()), c64(tm_est), c64(theta),
                                    f32(Id), (LAM, PS, NA, 20 * LAM),
                                    torch.from_numpy(phi).to(dev()), nf, nf)
    assert abs(g.item() - gref) <= 1e-9 * gref
    assert relerr(grad.cpu().numpy(), grad_ref) < 1e-9


@pytest.mark.parametrize("nf1,nf2,NA", [(64, 64, 0.22), (16, 8, 0.6), (2, 4, 0.9), (8, 8, 0.95), (128, 32, 0.1)])
def test_band_matches_full_path(ctx, nf1, nf2, NA):
    # the pruned evaluation against the full-FFT one on the same inputs (both also against the oracle above)
    print(f"band vs full nf1={nf1} nf2={nf2} NA={NA}", flush=True)
    g = np.random.default_rng(nf1 * 7 + nf2)
    P = min(nf1 * nf2, 300)
    pix = np.sort(g.choice(nf1 * nf2, P, replace=False))
    tm_est = tm_synth.tm_iid(P, 40, tm_synth.rng(955, 1)).astype(np.complex64)
    theta = tm_synth.defocus_phases(6, 40, tm_synth.rng(955, 4)).astype(np.complex64)
    Id = (np.abs(g.standard_normal((6, 2 * nf1, 2 * nf2))) * 1e3).astype(np.float32)
    phi = torch.from_numpy(g.random(P) * 2 * np.pi).to(dev())
    args = (torch.from_numpy(pix.astype(np.int32)).to(dev()), c64(tm_est), c64(theta), f32(Id),
            (LAM, PS, NA, 20 * LAM), phi, nf1, nf2)
    out = {}
    for on in (True, False):
        tm.tm_phase_set_band(ctx, on)
        gv, grad = tm.tm_phase_objective(ctx, *args)
        out[on] = (gv.item(), grad.cpu().numpy())
    tm.tm_phase_set_band(ctx, True)
    assert abs(out[True][0] - out[False][0]) <= 1e-11 * abs(out[False][0])
    assert relerr(out[True][1], out[False][1]) < 1e-11


def test_noiseless_offsets_recovered(ctx):
    nf, P, N, Nd = 16, 40, 24, 12
    pix, tm_est, theta, Id, phi_true, mdl = build(nf, P, N, Nd, 0.6, 0.6, cfg=951)
    phi_o, hist = df.lbfgs_phase(mdl, Id.astype(np.float64), np.zeros(P), 200)
    phi = torch.zeros(P, dtype=torch.float64, device=dev())
    g = tm.tm_phase_offset_correct(ctx, torch.from_numpy(pix.astype(np.int32)).to(dev()), c64(tm_est), c64(theta),
                                   f32(Id), (LAM, PS, 0.6, 20 * LAM), phi, nf, nf, iters=200, m=5)
    err = df.circular_offset_error(phi.cpu().numpy(), phi_true)
    err_o = df.circular_offset_error(phi_o, phi_true)
    print("gpu max err", np.max(np.abs(err)), "oracle", np.max(np.abs(err_o)), "g", g, hist[-1])
    # the data are FP32-rounded images of the exact model, so the floor is that rounding
    assert np.max(np.abs(err)) < 1e-5
    assert np.max(np.abs(err - err_o)) < 1e-5


@pytest.mark.parametrize("iters", [1, 2, 3, 6, 12])
def test_iterations_follow_the_oracle(ctx, iters):
    # the device line search (growing step, kept trial, halving) and the
    # compact L-BFGS direction take the oracle's steps iteration by iteration
    nf, P, N, Nd = 16, 40, 24, 12
    pix, tm_est, theta, Id, phi_true, mdl = build(nf, P, N, Nd, 0.6, 0.6, cfg=957, noise=1e4)
    trace = []
    phi_o, hist = df.lbfgs_phase(mdl, Id.astype(np.float64), np.zeros(P), iters, trace=trace)
    phi = torch.zeros(P, dtype=torch.float64, device=dev())
    g = tm.tm_phase_offset_correct(ctx, torch.from_numpy(pix.astype(np.int32)).to(dev()), c64(tm_est), c64(theta),
                                   f32(Id), (LAM, PS, 0.6, 20 * LAM), phi, nf, nf, iters=iters, m=5)
    print(f"iters {iters}: {len(trace)} oracle trials, steps {[t[0] for t in trace][:8]}", flush=True)
    assert np.max(np.abs(phi.cpu().numpy() - phi_o)) <= 1e-9 * max(1.0, np.max(np.abs(phi_o)))
    assert abs(g - hist[-1]) <= 1e-11 * hist[-1]
    # the same trials: one evaluation at the start plus one per trial point
    assert tm.tm_phase_last_counts(ctx) == (iters, 1 + len(trace))


def test_full_size_iterations_follow_the_oracle(ctx):
    # the benchmark's phase solve (2286 pixels of a 64 x 64 field, 8192 modes,
    # 50 defocus images, NA 0.22, memory 1) for its first iterations
    nf, P, N, Nd, NA = 64, 2286, 8192, 50, 0.22
    pix, tm_est, theta, Id, phi_true, mdl = build(nf, P, N, Nd, NA, 0.22, cfg=960, noise=1e4)
    for iters in (1, 4):
        trace = []
        phi_o, hist = df.lbfgs_phase(mdl, Id.astype(np.float64), np.zeros(P), iters, m=1, trace=trace)
        phi = torch.zeros(P, dtype=torch.float64, device=dev())
        g = tm.tm_phase_offset_correct(ctx, torch.from_numpy(pix.astype(np.int32)).to(dev()), c64(tm_est),
                                       c64(theta), f32(Id), (LAM, PS, NA, 20 * LAM), phi, nf, nf, iters=iters, m=1)
        print(f"full-size phase iters {iters}: trials {[t[0] for t in trace]}", flush=True)
        assert np.max(np.abs(phi.cpu().numpy() - phi_o)) <= 1e-9 * max(1.0, np.max(np.abs(phi_o)))
        assert abs(g - hist[-1]) <= 1e-11 * hist[-1]
        assert tm.tm_phase_last_counts(ctx) == (iters, 1 + len(trace))


def test_rejects_bad_pixels(ctx):
    nf, P, N, Nd = 16, 40, 24, 12
    pix, tm_est, theta, Id, _, _ = build(nf, P, N, Nd, 0.6, 0.6, cfg=952)
    bad = pix.astype(np.int32).copy()
    bad[3] = nf * nf + 5
    with pytest.raises(tm.TMError, match="outside the field grid"):
        tm.tm_phase_objective(ctx, torch.from_numpy(bad).to(dev()), c64(tm_est), c64(theta), f32(Id),
                              (LAM, PS, 0.6, 20.0), torch.zeros(P, dtype=torch.float64, device=dev()), nf, nf)
    bad[3] = bad[4]
    with pytest.raises(tm.TMError, match="repeats"):
        tm.tm_phase_objective(ctx, torch.from_numpy(bad).to(dev()), c64(tm_est), c64(theta), f32(Id),
                              (LAM, PS, 0.6, 20.0), torch.zeros(P, dtype=torch.float64, device=dev()), nf, nf)


def test_zero_iterations_and_repeated_counts(ctx):
    # iters = 0 evaluates the start only (phi unchanged, g = g(phi0)); repeated
    # solves of the same size report the same counts (the replay batch is sized
    # from the previous solve's evaluations)
    nf, P, N, Nd = 16, 40, 24, 12
    pix, tm_est, theta, Id, _, mdl = build(nf, P, N, Nd, 0.6, 0.6, cfg=959, noise=1e4)
    args = (torch.from_numpy(pix.astype(np.int32)).to(dev()), c64(tm_est), c64(theta), f32(Id),
            (LAM, PS, 0.6, 20 * LAM))
    phi0 = np.random.default_rng(959).random(P)
    phi = torch.from_numpy(phi0.copy()).to(dev())
    g = tm.tm_phase_offset_correct(ctx, *args, phi, nf, nf, iters=0, m=5)
    assert tm.tm_phase_last_counts(ctx) == (0, 1)
    assert np.array_equal(phi.cpu().numpy(), phi0)
    assert abs(g - mdl.objective(Id.astype(np.float64), phi0)[0]) <= 1e-9 * g
    counts = []
    for _ in range(3):
        phi = torch.zeros(P, dtype=torch.float64, device=dev())
        tm.tm_phase_offset_correct(ctx, *args, phi, nf, nf, iters=15, m=5)
        counts.append(tm.tm_phase_last_counts(ctx))
    assert counts[0] == counts[1] == counts[2] and counts[0][0] == 15 and counts[0][1] >= 16


def test_solve_rejects_bad_pixels_on_the_device(ctx):
    # tm_phase_offset_correct checks pix on the device: an index outside the
    # grid or a pixel two rows share is reported when the call returns, phi is
    # left as it was, and the next solve on the same context is unaffected
    nf, P, N, Nd = 16, 40, 24, 12
    pix, tm_est, theta, Id, _, _ = build(nf, P, N, Nd, 0.6, 0.6, cfg=958)
    args = (c64(tm_est), c64(theta), f32(Id), (LAM, PS, 0.6, 20 * LAM))

    def solve(c, p, iters=20):
        phi = torch.full((P,), 0.25, dtype=torch.float64, device=dev())
        g = tm.tm_phase_offset_correct(c, torch.from_numpy(p.astype(np.int32)).to(dev()), *args, phi, nf, nf,
                                       iters=iters, m=5)
        return phi.cpu().numpy(), g

    good, g_good = solve(ctx, pix)
    for bad, msg in (((7, nf * nf + 5), r"pix\[7\]=\d+ outside the field grid"), ((9, -1), r"pix\[9\]=-1 outside"),
                     ((11, None), r"pix\[5\]=\d+ repeats a pixel")):
        q = pix.astype(np.int64).copy()
        if bad[1] is None:
            q[bad[0]] = q[5]
        else:
            q[bad[0]] = bad[1]
        for iters in (0, 20):
            phi = torch.full((P,), 0.25, dtype=torch.float64, device=dev())
            with pytest.raises(tm.TMError, match=msg):
                tm.tm_phase_offset_correct(ctx, torch.from_numpy(q.astype(np.int32)).to(dev()), *args, phi, nf, nf,
                                           iters=iters, m=5)
            assert torch.all(phi == 0.25)
    again, g_again = solve(ctx, pix)
    assert np.array_equal(good, again) and g_good == g_again
    c2 = tm.Context(0)
    try:
        fresh, g_fresh = solve(c2, pix)
    finally:
        c2.close()
    assert np.array_equal(good, fresh) and g_good == g_fresh


@pytest.mark.parametrize("nf1,nf2,P,N,Nd", [(8, 16, 50, 24, 3), (32, 4, 60, 16, 2), (2, 2, 3, 8, 2),
                                            (256, 4, 40, 8, 2), (4, 256, 40, 8, 2)])
def test_rectangular_grids_images_objective(ctx, nf1, nf2, P, N, Nd):
    # non-square field grids, line lengths from 2 to 512 (one line per workgroup)
    print(f"rectangular nf1={nf1} nf2={nf2} P={P}", flush=True)
    g = np.random.default_rng(nf1 * 1000 + nf2)
    pix = np.sort(g.choice(nf1 * nf2, P, replace=False))
    tm_est = tm_synth.tm_iid(P, N, tm_synth.rng(953, 1)).astype(np.complex64)
    theta = tm_synth.defocus_phases(Nd, N, tm_synth.rng(953, 4)).astype(np.complex64)
    mdl = df.DefocusModel(tm_est.astype(np.complex128), theta.astype(np.complex128), pix, nf1, nf2, LAM, PS, 0.6,
                          20 * LAM)
    phi = g.random(P) * 2 * np.pi
    pix_d = torch.from_numpy(pix.astype(np.int32)).to(dev())
    img = tm.tm_defocus_forward(ctx, pix_d, c64(tm_est), c64(theta), (LAM, PS, 0.6, 20 * LAM),
                                torch.from_numpy(phi).to(dev()), nf1, nf2)
    ref = mdl.images(phi)
    assert img.shape == ref.shape
    assert relerr(img.cpu().numpy(), ref) < 1e-6
    Id = (ref * (1 + 0.05 * g.standard_normal(ref.shape))).astype(np.float32)
    gref, grad_ref = mdl.objective(Id.astype(np.float64), phi)
    gv, grad = tm.tm_phase_objective(ctx, pix_d, c64(tm_est), c64(theta), f32(Id), (LAM, PS, 0.6, 20 * LAM),
                                     torch.from_numpy(phi).to(dev()), nf1, nf2)
    assert abs(gv.item() - gref) <= 1e-9 * gref
    assert relerr(grad.cpu().numpy(), grad_ref) < 1e-9


def test_ftol_stops_early(ctx):
    # a relative-decrease tolerance ends the solve after an accepted iteration:
    # an enormous one after the first (same result as iters=1), a tiny one
    # still at the converged offsets
    nf, P, N, Nd = 16, 40, 24, 12
    pix, tm_est, theta, Id, phi_true, mdl = build(nf, P, N, Nd, 0.6, 0.6, cfg=954)
    args = (torch.from_numpy(pix.astype(np.int32)).to(dev()), c64(tm_est), c64(theta), f32(Id),
            (LAM, PS, 0.6, 20 * LAM))

    def solve(iters, ftol):
        phi = torch.zeros(P, dtype=torch.float64, device=dev())
        g = tm.tm_phase_offset_correct(ctx, *args, phi, nf, nf, iters=iters, m=5, ftol=ftol)
        return phi.cpu().numpy(), g

    one, g1 = solve(1, 0.0)
    big, gb = solve(200, 1e300)
    assert np.array_equal(one, big) and g1 == gb
    tight, gt = solve(200, 1e-14)
    assert np.max(np.abs(df.circular_offset_error(tight, phi_true))) < 1e-5
    with pytest.raises(tm.TMError, match="ftol"):
        solve(10, -1.0)


def test_repeated_solves_reuse_the_captured_iteration(ctx):
    # the captured iteration is kept between calls while its inputs' addresses
    # and sizes are unchanged: repeated and changed solves equal fresh contexts'
    nf, P, N, Nd = 16, 40, 24, 12
    pix, tm_est, theta, Id, phi_true, mdl = build(nf, P, N, Nd, 0.6, 0.6, cfg=956, noise=1e4)
    pix_d, tm_d, th_d, Id_d = (torch.from_numpy(pix.astype(np.int32)).to(dev()), c64(tm_est), c64(theta), f32(Id))
    opt = (LAM, PS, 0.6, 20 * LAM)

    def solve(c, iters, Idt=Id_d):
        phi = torch.zeros(P, dtype=torch.float64, device=dev())
        g = tm.tm_phase_offset_correct(c, pix_d, tm_d, th_d, Idt, opt, phi, nf, nf, iters=iters, m=5)
        return phi.cpu().numpy(), g

    a1, g1 = solve(ctx, 50)
    a2, g2 = solve(ctx, 50)
    assert np.array_equal(a1, a2) and g1 == g2
    Id_d.mul_(1.01)  # same address, new contents
    b1, _ = solve(ctx, 50)
    b2, _ = solve(ctx, 30)
    fresh = tm.Context(0)
    try:
        fb1, _ = solve(fresh, 50)
        fb2, _ = solve(fresh, 30)
    finally:
        fresh.close()
    assert np.array_equal(b1, fb1) and np.array_equal(b2, fb2)
    assert not np.array_equal(a1, b1)


@pytest.mark.parametrize("nf,P,N,Nd,NA,noise", [(16, 40, 24, 12, 0.6, 1e4), (32, 512, 1024, 50, 0.3, 1e4)])
def test_async_solve_equals_the_synchronous_one(ctx, nf, P, N, Nd, NA, noise):
    # the stream-ordered solve, given the evaluations the synchronous solve
    # reported (or more), computes the same offsets and objective bit for bit
    # and records the same counts; with fewer it records an unfinished solve
    pix, tm_est, theta, Id, _, _ = build(nf, P, N, Nd, NA, 0.6, cfg=963, noise=noise)
    args = (torch.from_numpy(pix.astype(np.int32)).to(dev()), c64(tm_est), c64(theta), f32(Id),
            (LAM, PS, NA, 20 * LAM))
    phi_s = torch.zeros(P, dtype=torch.float64, device=dev())
    g_s = tm.tm_phase_offset_correct(ctx, *args, phi_s, nf, nf, iters=25, m=5)
    it, ev = tm.tm_phase_last_counts(ctx)
    assert it == 25 and ev > 25
    other = tm.Context(0)
    side = torch.cuda.Stream()
    try:
        for c in (ctx, other):
            for evals in (ev, ev + 13, ev + 20):
                rec = torch.full((8,), -1.0, dtype=torch.float64, device=dev())
                phi = torch.zeros(P, dtype=torch.float64, device=dev())
                side.wait_stream(torch.cuda.current_stream())
                with torch.cuda.stream(side):
                    tm.tm_phase_offset_correct_async(c, *args, phi, nf, nf, rec, evals, iters=25, m=5)
                torch.cuda.current_stream().wait_stream(side)
                r = rec.cpu().numpy()
                assert torch.equal(phi, phi_s)
                assert r[0] == g_s and (r[1], r[2], r[3], r[4]) == (25, ev, 1, 0)
            assert tm.tm_phase_last_counts(ctx) == (it, ev)  # the synchronous call's counts
        for evals in (1, ev // 2, ev - 1):
            rec = torch.zeros(8, dtype=torch.float64, device=dev())
            phi = torch.zeros(P, dtype=torch.float64, device=dev())
            tm.tm_phase_offset_correct_async(ctx, *args, phi, nf, nf, rec, evals, iters=25, m=5)
            r = rec.cpu().numpy()
            assert r[3] == 0 and r[2] == evals + 1 and r[1] < 25 and r[4] == 0
        # then the synchronous solve again: the same result
        phi = torch.zeros(P, dtype=torch.float64, device=dev())
        assert tm.tm_phase_offset_correct(ctx, *args, phi, nf, nf, iters=25, m=5) == g_s
        assert torch.equal(phi, phi_s)
    finally:
        other.close()


def test_async_solve_records_bad_pixels_and_rejects_bad_arguments(ctx):
    nf, P, N, Nd = 16, 40, 24, 12
    pix, tm_est, theta, Id, _, mdl = build(nf, P, N, Nd, 0.6, 0.6, cfg=964)
    rest = (c64(tm_est), c64(theta), f32(Id), (LAM, PS, 0.6, 20 * LAM))
    pix_d = torch.from_numpy(pix.astype(np.int32)).to(dev())
    for row, val, flag, slot in ((7, nf * nf + 5, 1, 5), (11, None, 2, 6)):
        q = pix.astype(np.int64).copy()
        q[row] = q[5] if val is None else val
        for iters in (0, 20):
            rec = torch.zeros(8, dtype=torch.float64, device=dev())
            phi = torch.full((P,), 0.25, dtype=torch.float64, device=dev())
            tm.tm_phase_offset_correct_async(ctx, torch.from_numpy(q.astype(np.int32)).to(dev()), *rest, phi, nf, nf,
                                             rec, 30, iters=iters, m=5)
            r = rec.cpu().numpy()
            assert r[4] == flag and r[slot] == (row if val is not None else 5) and r[3] == 1
            assert torch.all(phi == 0.25)
    # iters = 0: the start point's objective, one evaluation, evals ignored
    rec = torch.zeros(8, dtype=torch.float64, device=dev())
    phi0 = np.random.default_rng(964).random(P)
    phi = torch.from_numpy(phi0.copy()).to(dev())
    tm.tm_phase_offset_correct_async(ctx, pix_d, *rest, phi, nf, nf, rec, 0, iters=0, m=5)
    r = rec.cpu().numpy()
    assert (r[1], r[2], r[3], r[4]) == (0, 1, 1, 0)
    assert abs(r[0] - mdl.objective(Id.astype(np.float64), phi0)[0]) <= 1e-9 * r[0]
    assert np.array_equal(phi.cpu().numpy(), phi0)
    phi = torch.zeros(P, dtype=torch.float64, device=dev())
    for evals in (0, -1, 40 * 20 + 3):
        with pytest.raises(tm.TMError, match="evals"):
            tm.tm_phase_offset_correct_async(ctx, pix_d, *rest, phi, nf, nf, rec, evals, iters=20, m=5)
    for bad in (torch.zeros(6, dtype=torch.float64, device=dev()), torch.zeros(8, dtype=torch.float32, device=dev()),
                torch.zeros(8, dtype=torch.float64)):
        with pytest.raises(tm.TMError, match="rec"):
            tm.tm_phase_offset_correct_async(ctx, pix_d, *rest, phi, nf, nf, bad, 30, iters=20, m=5)


def test_async_solves_overlap_on_two_streams(ctx):
    # two problems solved at once, each on its own context and stream (the
    # pattern of a pipelined caller): each equals its synchronous solve
    nf, P, N, Nd, NA = 32, 512, 1024, 50, 0.3
    probs = []
    for cfg in (965, 966):
        pix, tm_est, theta, Id, _, _ = build(nf, P, N, Nd, NA, 0.6, cfg=cfg, noise=1e4)
        probs.append((torch.from_numpy(pix.astype(np.int32)).to(dev()), c64(tm_est), c64(theta), f32(Id),
                      (LAM, PS, NA, 20 * LAM)))
    sync = []
    for args in probs:
        phi = torch.zeros(P, dtype=torch.float64, device=dev())
        g = tm.tm_phase_offset_correct(ctx, *args, phi, nf, nf, iters=30, m=1)
        sync.append((phi, g, tm.tm_phase_last_counts(ctx)))
    ctxs = [tm.Context(0), tm.Context(0)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    try:
        recs = torch.zeros((2, 8), dtype=torch.float64, device=dev())
        phis = [torch.zeros(P, dtype=torch.float64, device=dev()) for _ in range(2)]
        for s in streams:
            s.wait_stream(torch.cuda.current_stream())
        for k in range(2):
            with torch.cuda.stream(streams[k]):
                tm.tm_phase_offset_correct_async(ctxs[k], *probs[k], phis[k], nf, nf, recs[k], sync[k][2][1] + 2,
                                                 iters=30, m=1)
        for s in streams:
            torch.cuda.current_stream().wait_stream(s)
        r = recs.cpu().numpy()
        for k in range(2):
            assert torch.equal(phis[k], sync[k][0])
            assert r[k, 0] == sync[k][1] and (r[k, 1], r[k, 2], r[k, 3], r[k, 4]) == (30, sync[k][2][1], 1, 0)
        assert not torch.equal(phis[0], phis[1])
    finally:
        for c in ctxs:
            c.close()
