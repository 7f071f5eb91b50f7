"""Benchmark: TM rows/s to fidelity 0.99 on one MI355X.

Workload (the paper-scale configuration): N = 8192 input modes on a 128 x 64
grid, P = 2286 output pixels (the pixels of a 64 x 64 grid nearest its
centre), band-limited speckle TM (pupil 0.22 of the grid Nyquist), K = 4
random-phase masks (32768 intensities per row), Poisson noise at a mean of
1e4 photons per pixel, FP32 intensities; 50 defocus images (128 x 128) at
z = 20 wavelengths for the phase-offset step. All inputs are seeded and
synthetic (the paper's measured data are not available).

A step is one pass of the whole path over the batch: truncated spectral
start (Lanczos steps on the weighted operator, Ritz vector), cyclic
error-reduction sweeps up to the count at which the mean per-row fidelity
first reaches 0.99, the FP64 acceptance residual, and the per-row
phase-offset correction from the defocus images, run for the iteration count
at which the offsets have converged (both counts found by untimed
instrumented runs). value = P / step time. --start and --solver select the
heavy-ball start and the averaged (Nesterov) error reduction instead.

Also printed in the same JSON line: the roofline of the dominant kernel
(the fused Lanczos-step kernel, event-timed live on the library's stream)
and of the solver's kernel, counter-measured HBM traffic while the kernel
sources match the committed summary, the variants (L-BFGS, learned start,
foci, dense comparator, preprocessing, uneven batch), and the FP64 oracle
timed on the host's cores over a bounded sample of rows (`cpu_baseline`).
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 157.3  # published vector FP32 (packed) peak; 78.6 without packed math
BF16_MFMA_PEAK_TFLOPS = 2500.0  # published dense BF16 matrix peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch-start", choices=["spectral", "lanczos"], default="lanczos",
                    help="spectral start of the uneven batch")
    ap.add_argument("--batch-spectral-iters", type=int, default=None,
                    help="spectral steps in the uneven batch (default 24 heavy-ball, 17 Lanczos)")
    ap.add_argument("--batch-spectral-tau", type=float, default=None,
                    help="truncation of the spectral weights in the uneven batch (default 2.5 heavy-ball, 3.0 Lanczos)")
    ap.add_argument("--start", choices=["spectral", "lanczos"], default="lanczos",
                    help="spectral start by heavy-ball power steps or by Lanczos steps")
    ap.add_argument("--spectral-iters", type=int, default=None,
                    help="steps of the spectral start (default 24 heavy-ball or 17 Lanczos)")
    ap.add_argument("--spectral-tau", type=float, default=None,
                    help="truncation of the spectral weights (default 2.5 heavy-ball, 3.0 Lanczos)")
    ap.add_argument("--spectral-momentum", type=float, default=0.99,
                    help="heavy-ball factor c of the spectral start")
    ap.add_argument("--spectral-lower", type=float, default=0.0,
                    help="lower end of the rest of the spectrum (fraction of lambda); -c: unshifted heavy ball")
    ap.add_argument("--phase-iters", type=int, default=200,
                    help="phase L-BFGS iterations (with --phase-auto: the reference count and upper bound)")
    ap.add_argument("--phase-auto", type=int, default=1,
                    help="1: use the smallest count (multiple of 5, from 20) whose offset spread is within 1%% of the "
                         "reference, found by an untimed run")
    ap.add_argument("--phase-m", type=int, default=1,
                    help="L-BFGS memory of the phase solve (1: as few iterations as 3..12 at this workload, and "
                         "the cheapest iteration)")
    ap.add_argument("--phase-ftol", type=float, default=0.0,
                    help="stop the phase solve after an accepted iteration lowering g by <= ftol * g")
    ap.add_argument("--max-iters", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--small", action="store_true", help="32x32 modes, 512 rows (quick check)")
    ap.add_argument("--er-iters", type=int, default=0, help="skip the instrumented search and use this count")
    ap.add_argument("--solver", choices=["er", "er_cyclic"], default="er_cyclic",
                    help="error reduction averaging the K mask projections (er, with --er-momentum) or taking "
                         "them one at a time (er_cyclic)")
    ap.add_argument("--er-momentum", type=float, default=0.8,
                    help="Nesterov factor of the error-reduction iterations (0: plain ER)")
    ap.add_argument("--batch-iters", type=int, default=None,
                    help="iterations in the uneven batch (default 30 for er; er_cyclic: 5 sweeps after the "
                         "Lanczos start, 6 after the heavy-ball start)")
    ap.add_argument("--no-lbfgs", action="store_true", help="skip the L-BFGS comparison")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-start variant")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven 12-TM batch")
    ap.add_argument("--no-preprocess", action="store_true", help="skip the camera-stack preprocessing")
    ap.add_argument("--no-foci", action="store_true", help="skip the foci power ratio")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense-probing comparator")
    ap.add_argument("--train-steps", type=int, default=150, help="training steps of the weighting network")
    ap.add_argument("--train-power-steps", type=int, default=20, help="power steps per training loss")
    ap.add_argument("--learned-rho-fallback", type=float, default=0.0,
                    help="FP64 residual above which a row of the learned form is redone from the plain start in the "
                         "timed learned form (0: no fallback; the fallback forms are reported as variants)")
    ap.add_argument("--profile-lbfgs", type=int, default=0, metavar="ITERS",
                    help="only run one L-BFGS retrieval of ITERS iterations on the workload (for counter runs)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: time every compiled launch configuration of the Lanczos and cyclic ER kernels for the "
                         "grid before the timed steps and use the fastest; 0: the default configuration")
    ap.add_argument("--pipeline", type=int, default=1,
                    help="1: overlap step i's phase solve (second stream) with step i+1's retrieval; 0: serial steps")
    ap.add_argument("--config", type=int, default=None,
                    help="use this launch configuration (tm_config_info) instead of tuning (profiling runs)")
    ap.add_argument("--gemm-probe", action="store_true",
                    help="only time the network's BF16 MFMA GEMM at the shapes of one training step (cfg4 network)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 512 MiB device-to-device 5 times (reference for HBM byte counters)")
    ap.add_argument("--trace-summary", metavar="DIR",
                    help="kernel calls and durations inside the timed region of a rocprofv3 --kernel-trace "
                         "--marker-trace run (no GPU)")
    ap.add_argument("--pmc-summary", nargs=5, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR",
                                                        "OUT"),
                    help="summarise rocprofv3 FETCH_SIZE/WRITE_SIZE CSVs into the traffic file (no GPU)")
    args = ap.parse_args()
    if args.batch_iters is None:  # each TM's mean fidelity reaches 0.99 (GPU sweep)
        args.batch_iters = 30 if args.solver == "er" else (5 if args.batch_start == "lanczos" else 6)
    if args.batch_spectral_iters is None:
        args.batch_spectral_iters = 17 if args.batch_start == "lanczos" else 24
    if args.batch_spectral_tau is None:
        args.batch_spectral_tau = 3.0 if args.batch_start == "lanczos" else 2.5
    if args.spectral_tau is None:
        args.spectral_tau = 3.0 if args.start == "lanczos" else 2.5
    if args.spectral_iters is None:
        args.spectral_iters = 17 if args.start == "lanczos" else 24
    return args


KERNEL_SOURCES = ["fft_core.hpp", "row_kernels.hpp", "grid_inst.hip", "grids.hpp"]
LBFGS_SOURCES = ["lbfgs_kernels.hip", "lbfgs.hpp", "row_kernels.hpp", "fft_core.hpp", "grids.hpp"]  # with what it includes
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_2286x8192.json")
PHASE_EVAL_MARGIN = 2  # evaluations queued beyond the synchronous solve's count (the extra ones return at once)
PIPE_BUFFERS = 3  # row buffers of the pipelined steps: retrieval i reuses the buffer of phase solve i - 3
TIMED_RANGE = "bench timed steps"


def sources_digest(files=None):
    """SHA-256 over the kernels' sources (default: the fused row kernels):
    counter-measured traffic is used only while these are unchanged."""
    import hashlib
    h = hashlib.sha256()
    for f in files or KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2302_13524_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def plan_tag(L1, L2, cfg):
    """The Plan<...> of the row kernels that launch configuration cfg runs
    (as rocprofv3 names them): eight values per thread with bit 2, the digit
    order of bit 1."""
    return f"Plan<{L1}, {L2}, {3 if cfg & 2 else -1}, {cfg & 1}>"


def measured_traffic(P, N, plan=None):
    """HBM bytes per launch of the spectral and ER kernels from the committed
    FETCH_SIZE / WRITE_SIZE counter summary, scaled by the counters' reading
    for a device copy of known size; None when absent or taken on other
    sources; a row kernel's entry only when its counters were taken on `plan`
    (the launch configuration's Plan<...>), if given."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        d = json.load(fh)
    if d.get("P") != P or d.get("N") != N:
        return None
    fs = d["copy"]["bytes"] / 1024 / d["copy"]["fetch_kib"]
    ws = d["copy"]["bytes"] / 1024 / d["copy"]["write_kib"]
    ok = {"row": d.get("sources_sha256") == sources_digest(),
          "lbfgs": d.get("lbfgs_sources_sha256") == sources_digest(LBFGS_SOURCES)}
    return {k: int(round((v["fetch_kib"] * fs + v["write_kib"] * ws) * 1024)) for k, v in d["kernels"].items()
            if ok["lbfgs" if k.startswith("lbfgs") else "row"]
            and (plan is None or k.startswith("lbfgs") or v.get("plan") == plan)}


def pmc_summary(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, out):
    """Write the traffic summary from rocprofv3 counter CSVs (FETCH_SIZE run,
    WRITE_SIZE run, and the same two for --copy-probe): per-dispatch averages
    in KiB for the spectral and ER row kernels at this workload."""
    import csv
    import glob

    def per_kernel(d, counter):
        acc = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r.get("Counter_Name") != counter:
                    continue
                acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}

    def pick(tab, mode):
        # the launch configuration's kernels (default or autotuned plan) of this mode, with and
        # without sums; where several plans ran, the one with the most dispatches
        plans = {}
        for k in tab:
            m = re.match(r"void tmk::row_kernel(?:_w)?<tmk::(Plan<7, 6, -?\d+, \d+>), (\d+), float, ", k)
            if m and int(m.group(2)) == mode:
                plans.setdefault(m.group(1), []).append(tab[k])
        plan = max(plans, key=lambda q: sum(c for _, c in plans[q]))
        vals = plans[plan]
        n = sum(c for _, c in vals)
        return sum(v * c for v, c in vals) / n, n, plan

    f, w = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    cf, cw = per_kernel(copy_fetch_dir, "FETCH_SIZE"), per_kernel(copy_write_dir, "WRITE_SIZE")
    big = max(cf, key=lambda k: cf[k][0])
    res = {"P": 2286, "N": 8192, "sources_sha256": sources_digest(),
           "lbfgs_sources_sha256": sources_digest(LBFGS_SOURCES),
           "copy": {"kernel": big, "bytes": 512 * 2**20, "fetch_kib": cf[big][0], "write_kib": cw[big][0]},
           "kernels": {}}
    for key, mode in (("spectral", 5), ("er", 3), ("er_cyclic", 12), ("lanczos", 13)):
        if not any(f", {mode}, float, " in k for k in f):
            continue
        fv, fn, plan = pick(f, mode)
        wv, wn, _ = pick(w, mode)
        res["kernels"][key] = {"fetch_kib": fv, "write_kib": wv, "dispatches": [fn, wn], "plan": plan}

    def pick_name(tab, frag):
        keys = [k for k in tab if frag in k]
        vals = [tab[k] for k in keys]
        n = sum(c for _, c in vals)
        return (sum(v * c for v, c in vals) / n, n) if n else (None, 0)

    # the L-BFGS kernels (one --profile-lbfgs run: iterations with 0..m stored pairs, as in the timed leg)
    lb = {}
    for key, frag in (("lbfgs_dots", "k_dir_dots"), ("lbfgs_step", "k_step<")):
        fv, fn = pick_name(f, frag)
        wv, wn = pick_name(w, frag)
        if fv is not None and wv is not None:
            lb[key] = {"fetch_kib": fv, "write_kib": wv, "dispatches": [fn, wn]}
    if "lbfgs_dots" in lb:  # the direction's HBM pass (k_dir_solve reads only the partial sums)
        lb["lbfgs_direction"] = dict(lb["lbfgs_dots"])
    res["kernels"].update(lb)
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))


def trace_summary(d, top=16):
    """Per-kernel calls and average duration over the dispatches inside the
    bench's timed region, from a rocprofv3 run with --kernel-trace and
    --marker-trace (the region is the roctx range TIMED_RANGE; every kernel of
    the timed steps starts and ends inside it, since the range opens and closes
    on a synchronised device). Prints a markdown table."""
    import csv
    import glob

    def rows(pattern):
        out = []
        for f in glob.glob(os.path.join(d, "**", pattern), recursive=True):
            out += list(csv.DictReader(open(f)))
        return out

    marks = [r for r in rows("*marker_api_trace.csv") if any(TIMED_RANGE in str(v) for v in r.values())]
    if not marks:
        raise SystemExit(f"no '{TIMED_RANGE}' range in {d} (run rocprofv3 with --marker-trace)")
    lo = min(int(r["Start_Timestamp"]) for r in marks)
    hi = max(int(r["End_Timestamp"]) for r in marks)
    acc = {}
    for r in rows("*kernel_trace.csv"):
        a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        if a >= lo and b <= hi:
            acc.setdefault(r["Kernel_Name"], []).append((b - a) * 1e-3)
    tot = sum(sum(v) for v in acc.values())
    print(f"timed region {(hi - lo) * 1e-6:.3f} ms, {sum(len(v) for v in acc.values())} dispatches")
    print("| calls | avg (us) | total (ms) | share | kernel |\n|---:|---:|---:|---:|---|")
    for k, v in sorted(acc.items(), key=lambda kv: -sum(kv[1]))[:top]:
        name = k.replace("tmk::(anonymous namespace)::", "").replace("tmk::", "")
        print(f"| {len(v)} | {sum(v) / len(v):.2f} | {sum(v) * 1e-3:.3f} | {100 * sum(v) / tot:.1f}% | `{name[:100]}` |")
    return acc


def profile_lbfgs(iters):
    """One L-BFGS retrieval (Alg. 1, memory 5) of `iters` iterations on the
    benchmark workload from a spectral start, nothing else: the dispatch
    sequence the counter runs of the L-BFGS kernels read."""
    import torch

    import paper_2302_13524_amd as tm
    import tm_synth

    dev = torch.device("cuda:0")
    n1, n2, P, grid, pupil, K = 128, 64, 2286, 64, 0.22, 4
    N = n1 * n2
    pix = tm_synth.nearest_pixels(grid, P)
    masks = tm_synth.mask_phases(K, N, tm_synth.rng(3, 0))
    T = tm_synth.speckle_tm(N, grid, pupil, pix, tm_synth.rng(3, 1)).astype(np.complex64)
    v0 = tm_synth.random_start(P, N, np.ones(P), tm_synth.rng(3, 3)).astype(np.complex64)
    ctx = tm.Context(0)
    mk = torch.from_numpy(masks.astype(np.complex64)).to(dev)
    I = tm.tm_forward(ctx, mk, torch.from_numpy(T).to(dev), n1, n2, intensity=True)
    t = torch.from_numpy(v0).to(dev)
    tm.tm_retrieve(ctx, mk, I, t, n1, n2, tm.retrieve_opts("er", iters=0, start="lanczos", spectral_iters=17))
    tm.tm_retrieve(ctx, mk, I, t, n1, n2, tm.retrieve_opts("lbfgs", iters=iters, lbfgs_m=5), stats=False)
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps({"profile_lbfgs_iters": iters}))


def gemm_probe(reps=20):
    """The BF16 MFMA GEMM (tm_gemm_bf16: 128 x 128 tiles, double-buffered K
    steps) at the shapes of one training step of the start network
    (4096 -> 1024 -> 1024 -> 2048, batch 512: forward X W, backward dX = dY W^T
    and dW = X^T dY), and one 4096^3 product; each timed with events over
    `reps` launches on the current stream after one warm-up."""
    import torch

    import paper_2302_13524_amd as tm

    dev = torch.device("cuda:0")
    ctx = tm.Context(0)
    g = torch.Generator(device=dev)
    g.manual_seed(11)
    B, dims = 512, (4096, 1024, 1024, 2048)
    shapes = []
    for i in range(3):
        k, n = dims[i], dims[i + 1]
        shapes.append((f"fwd{i + 1} X W", B, n, k, False, False))
        shapes.append((f"bwd{i + 1} dY W^T", B, k, n, False, True))
        shapes.append((f"bwd{i + 1} X^T dY", k, n, B, True, False))
    shapes.append(("square 4096", 4096, 4096, 4096, False, False))
    out = []
    for name, M, N, K, ta, tb in shapes:
        A = torch.randn((K, M) if ta else (M, K), generator=g, device=dev).to(torch.bfloat16)
        Bm = torch.randn((N, K) if tb else (K, N), generator=g, device=dev).to(torch.bfloat16)
        tm.tm_gemm_bf16(ctx, A, Bm, ta, tb)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            tm.tm_gemm_bf16(ctx, A, Bm, ta, tb)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tf = 2.0 * M * N * K / (ms * 1e-3) / 1e12
        out.append({"gemm": name, "M": M, "N": N, "K": K, "ms": round(ms, 5), "TFLOPs": round(tf, 1),
                    "frac_bf16_peak": round(tf / BF16_MFMA_PEAK_TFLOPS, 4)})
    ctx.close()
    print(json.dumps({"gemm_probe": out}))


def copy_probe():
    import torch
    a = torch.empty(512 * 2**20 // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": a.numel() * 4, "copies": 5}))


def main():
    args = parse()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary)
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.gemm_probe:
        gemm_probe()
        return
    if args.profile_lbfgs:
        profile_lbfgs(args.profile_lbfgs)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); rows are independent problems, so "
              "more GPUs would each run this same kernel on P/G rows.", file=sys.stderr)
        sys.exit(2)
    pool = None if args.no_cpu_baseline else cpu_pool()  # host workers, started before the GPU is touched
    import torch

    import paper_2302_13524_amd as tm
    import tm_synth

    dev = torch.device("cuda:0")
    if args.small:
        n1, n2, P, grid, pupil, nf = 32, 32, 512, 32, 0.3, 32
        cfg_id = 2
    else:
        n1, n2, P, grid, pupil, nf = 128, 64, 2286, 64, 0.22, 64
        cfg_id = 3
    K, N, Nd = 4, n1 * n2, 50
    NA, lam, ps, z = pupil, 1.0, 0.5, 20.0
    workload = f"{P}x{N} TM ({n1}x{n2} modes), K={K}, speckle pupil {pupil}, Poisson 1e4, FP32 I; " \
               f"{Nd} defocus images {2*nf}x{2*nf}"

    t0 = time.perf_counter()
    pix = tm_synth.nearest_pixels(grid, P)
    masks = tm_synth.mask_phases(K, N, tm_synth.rng(cfg_id, 0))
    T = tm_synth.speckle_tm(N, grid, pupil, pix, tm_synth.rng(cfg_id, 1)).astype(np.complex64)
    v0 = tm_synth.random_start(P, N, np.ones(P), tm_synth.rng(cfg_id, 3)).astype(np.complex64)
    theta = tm_synth.defocus_phases(Nd, N, tm_synth.rng(cfg_id, 4)).astype(np.complex64)
    log(f"host synthesis {time.perf_counter() - t0:.1f}s")

    ctx = tm.Context(0)
    mk = torch.from_numpy(masks.astype(np.complex64)).to(dev)
    Tt = torch.from_numpy(T).to(dev)
    v0t = torch.from_numpy(v0).to(dev)
    th = torch.from_numpy(theta).to(dev)
    pixt = torch.from_numpy(pix.astype(np.int32)).to(dev)
    optics = (lam, ps, NA, z)

    # intensities: clean images by the forward model, shot noise drawn on the host (seeded). With the
    # CPU baseline on, the oracle's FP64 forward models make them (host workers), so that the GPU and the
    # oracle see the same FP32 inputs and their results can be compared row by row; otherwise the GPU's.
    if pool is not None:
        Ic, Idc = oracle_inputs(pool, masks, T, n1, n2, theta, pix, nf, optics)
        log(f"oracle forward models {time.perf_counter() - t0:.1f}s")
    else:
        Ic = tm.tm_forward(ctx, mk, Tt, n1, n2, intensity=True).cpu().numpy()
        Idc = tm.tm_defocus_forward(ctx, pixt, Tt, th, optics, torch.zeros(P, dtype=torch.float64, device=dev),
                                    nf, nf).cpu().numpy()
    I_np = tm_synth.poisson_counts(Ic.astype(np.float64), 1e4, tm_synth.rng(cfg_id, 2)).astype(np.float32)
    del Ic
    It = torch.from_numpy(I_np).to(dev)
    Id_np = tm_synth.poisson_counts(Idc.astype(np.float64), 1e4, tm_synth.rng(cfg_id, 5)).astype(np.float32)
    Idt = torch.from_numpy(Id_np).to(dev)
    log(f"inputs ready {time.perf_counter() - t0:.1f}s")

    Tn = Tt / torch.linalg.vector_norm(Tt, dim=1, keepdim=True)

    # launch configuration of the Lanczos and cyclic ER kernels for this grid (untimed)
    tune = {"config": 0}
    if args.config is not None:
        tm.tm_set_config(ctx, n1, n2, args.config)
        tune = {"config": args.config}
    elif args.autotune:
        tune = tm.autotune(ctx, n1, n2, K, P, space="full", reps=5)
        log(f"autotune {n1}x{n2}: config {tune['config']} {tm.tm_config_info(n1, n2, tune['config'])}")

    def fidelity(t):
        c = torch.sum(torch.conj(t) * Tn, dim=1)
        return (c.abs() ** 2 / torch.sum(t.abs() ** 2, dim=1)).double()

    sp = args.spectral_iters

    solver = args.solver
    beta = args.er_momentum if solver == "er" else 0.0
    er_mode = 3 if solver == "er" else 12  # row-kernel mode of the solver's iteration

    def opts(method, iters, start=None):
        start = args.start if start is None else start
        return tm.retrieve_opts(method, iters=iters, start=start, spectral_iters=sp, spectral_tau=args.spectral_tau,
                                spectral_momentum=args.spectral_momentum,
                                spectral_lower=args.spectral_lower,
                                er_momentum=beta if method == "er" else 0.0)

    def sopts(iters, start=None):
        return opts(solver, iters, start) if solver != "er" else opts("er", iters, start)

    # ---- untimed instrumented run: iterations to mean fidelity 0.99 (each count run
    # from the start, since the momentum iteration carries the previous iterate)
    t = v0t.clone()
    tm.tm_retrieve(ctx, mk, It, t, n1, n2, sopts(0))
    f_start = fidelity(t).mean().item()
    n_er = args.er_iters or None
    for it in range(1, 0 if n_er else args.max_iters + 1):
        t = v0t.clone()
        tm.tm_retrieve(ctx, mk, It, t, n1, n2, sopts(it), stats=False)
        if fidelity(t).mean().item() >= 0.99:
            n_er = it
            break
    if n_er is None:
        raise SystemExit(f"error reduction did not reach mean fidelity 0.99 in {args.max_iters} iterations")
    log(f"spectral start fidelity {f_start:.4f}; ER reaches 0.99 after {n_er} iterations")

    # ---- untimed instrumented run: phase iterations at which the offsets have converged (circular
    # spread over the rows at fidelity >= 0.99 within 1 % of the spread after phase_iters_max)
    t = v0t.clone()
    tm.tm_retrieve(ctx, mk, It, t, n1, n2, sopts(n_er), stats=False)
    good0 = fidelity(t) >= 0.99
    off_t = torch.angle(torch.sum(torch.conj(t) * Tt, dim=1)).double()

    def spread_of(iters):
        phi = torch.zeros(P, dtype=torch.float64, device=dev)
        tm.tm_phase_offset_correct(ctx, pixt, t, th, Idt, optics, phi, nf, nf, iters=iters, m=args.phase_m, ftol=args.phase_ftol)
        z = torch.exp(1j * (off_t - phi)[good0])
        return float(torch.sqrt(-2 * torch.log(torch.abs(z.mean()) + 1e-300)).item())

    n_ph = args.phase_iters
    if args.phase_auto:
        ref = spread_of(args.phase_iters)
        for k in range(20, args.phase_iters, 5):
            if spread_of(k) <= 1.01 * ref:
                n_ph = k
                break
        log(f"phase offsets converge after {n_ph} iterations (spread {ref:.5f} rad at {args.phase_iters})")
    n_lb = None
    for k in () if args.no_lbfgs else (5, 10, 15, 20, 25, 30, 40, 50, 70, 100):
        t = v0t.clone()
        tm.tm_retrieve(ctx, mk, It, t, n1, n2, opts("lbfgs", k), stats=False)
        if fidelity(t).mean().item() >= 0.99:
            n_lb = k
            break
    log(f"L-BFGS reaches 0.99 within {n_lb} iterations")
    n_la = None
    for k in () if args.no_lbfgs else (5, 8, 10, 12, 15, 20, 25, 30, 40, 50, 70, 100):
        t = v0t.clone()
        tm.tm_retrieve(ctx, mk, It, t, n1, n2, opts("lbfgs_amp", k), stats=False)
        if fidelity(t).mean().item() >= 0.99:
            n_la = k
            break
    log(f"amplitude L-BFGS reaches 0.99 within {n_la} iterations")

    def step(method=None, iters=n_er, phase=True):
        t = v0t.clone()
        raw = tm.tm_retrieve(ctx, mk, It, t, n1, n2, sopts(iters) if method is None else opts(method, iters))
        phi = None
        if phase:
            phi = torch.zeros(P, dtype=torch.float64, device=dev)
            tm.tm_phase_offset_correct(ctx, pixt, t, th, Idt, optics, phi, nf, nf, iters=n_ph, m=args.phase_m,
                                       ftol=args.phase_ftol)
        return t, raw, phi

    # Pipelined steps: the K steps are K independent TMs, so step i's phase solve (its own library
    # contexts, a second stream at the default priority) runs while step i + 1's retrieval runs on this
    # stream; PIPE_BUFFERS row buffers rotate, and a retrieval waits for the phase solve that last read its
    # buffer. Every step still runs its whole path inside the timed region. The phase solve's kernels are
    # latency-bound and small, so they fill the gaps of the retrieval's CU-filling kernels.
    # The phase solves are queued in their stream-ordered form, so the host never waits for one: each
    # queues the evaluations the synchronous solve of this problem took (every step repeats it) plus a
    # margin, and records whether it ended within them; every timed step's record is checked below.
    if args.pipeline:
        NB = PIPE_BUFFERS
        ctx_ph = [tm.Context(0) for _ in range(NB)]  # one per buffer: each keeps its captured phase graph
        s_ph = torch.cuda.Stream()
        tb = [v0t.clone() for _ in range(NB)]
        pb = [torch.zeros(P, dtype=torch.float64, device=dev) for _ in range(NB)]
        ev_r = [torch.cuda.Event() for _ in range(NB)]
        ev_p = [torch.cuda.Event() for _ in range(NB)]
        recs = torch.zeros((max(args.steps, args.warmup, NB), 8), dtype=torch.float64, device=dev)
        step()
        torch.cuda.synchronize()
        ph_budget = tm.tm_phase_last_counts(ctx)[1] + PHASE_EVAL_MARGIN

    def pipelined(k):
        main = torch.cuda.current_stream()
        raws = [None] * NB

        def retrieve(i):
            b = i % NB
            if i >= NB:
                main.wait_event(ev_p[b])  # step i - NB's phase solve has read this buffer
            tb[b].copy_(v0t)
            raws[b] = tm.tm_retrieve(ctx, mk, It, tb[b], n1, n2, sopts(n_er))
            ev_r[b].record(main)

        retrieve(0)
        for i in range(k):
            if i + 1 < k:
                retrieve(i + 1)
            b = i % NB
            with torch.cuda.stream(s_ph):
                s_ph.wait_event(ev_r[b])
                pb[b].zero_()
                tm.tm_phase_offset_correct_async(ctx_ph[b], pixt, tb[b], th, Idt, optics, pb[b], nf, nf, recs[i],
                                                 ph_budget, iters=n_ph, m=args.phase_m, ftol=args.phase_ftol)
                ev_p[b].record(s_ph)
        main.wait_event(ev_p[(k - 1) % NB])
        return tb[(k - 1) % NB], raws[(k - 1) % NB], pb[(k - 1) % NB]

    def serial_steps(k):
        out = None
        for _ in range(k):
            out = step()
        return out

    run_steps = pipelined if args.pipeline else serial_steps
    run_steps(max(args.warmup, PIPE_BUFFERS if args.pipeline else 0))  # with the pipeline: every phase context warm
    torch.cuda.synchronize()
    tm.tm_profile_enable(ctx, True)
    torch.cuda.synchronize()
    torch.cuda.nvtx.range_push(TIMED_RANGE)  # a roctx range: --trace-summary picks the timed region's kernels
    ts = time.perf_counter()
    t, raw, phi = run_steps(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - ts
    torch.cuda.nvtx.range_pop()
    er_ms, er_n = tm.tm_profile_query(ctx, er_mode)
    sp_mode = 13 if args.start == "lanczos" else 5  # row-kernel mode of the spectral start's step
    sp_ms, sp_n = tm.tm_profile_query(ctx, sp_mode)
    rs_ms, rs_n = tm.tm_profile_query(ctx, 7)
    tm.tm_profile_enable(ctx, False)
    ms_step = elapsed * 1e3 / args.steps
    if args.pipeline:
        rc = recs[:args.steps].cpu().numpy()
        if not (np.all(rc[:, 3] == 1) and np.all(rc[:, 4] == 0) and np.all(rc[:, 1] == rc[0, 1])):
            raise SystemExit(f"a pipelined phase solve did not end within {ph_budget} evaluations: {rc[:, :5]}")
        ph_it, ph_ev = int(rc[-1, 1]), int(rc[-1, 2])
    else:
        ph_it, ph_ev = tm.tm_phase_last_counts(ctx)
    log(f"phase solve of the last step: {ph_it} iterations, {ph_ev} objective evaluations")

    # component timings (retrieval only; phase correction only; L-BFGS variant)
    def timed(fn, reps=3):
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) * 1e3 / reps

    ret_ms = timed(lambda: step(phase=False))
    serial_kernels = None
    if args.pipeline:
        # the same steps one after another (no overlap): the step time, and the kernels' durations alone
        tm.tm_profile_enable(ctx, True)
        serial_ms = timed(step)
        sk = {m: tm.tm_profile_query(ctx, m) for m in (sp_mode, er_mode)}
        tm.tm_profile_enable(ctx, False)
        serial_kernels = {"spectral_avg": round(sk[sp_mode][0] / max(sk[sp_mode][1], 1), 5),
                          "er_avg": round(sk[er_mode][0] / max(sk[er_mode][1], 1), 5)}
    else:
        serial_ms = ms_step
    if args.pipeline:
        # the pipelined steps computed what the serial path computes
        t_s, _, phi_s = step()
        torch.cuda.synchronize()
        same_t = bool(torch.equal(t_s, t))
        same_phi = bool(torch.equal(phi_s, phi))
        if not (same_t and same_phi):
            raise SystemExit(f"pipelined steps differ from the serial path (t equal: {same_t}, phi equal: {same_phi})")
    roofline_lbfgs = None
    if n_lb:
        # the paper's Alg. 1: its direction kernels (dot products over the history, small solve) timed live
        # with HIP events on the library's stream, against HBM. Per row-iteration with c stored pairs and a
        # pending pair: read g, g_prev, s_new, write y_new, read the 2c history vectors: (1 + 3 + 2 c) 8 N
        # bytes (c = min(iteration, m), no pending pair at the first). The direction itself, d from g and
        # the history, is formed in the line search's row kernel ((2 + 2 c) 8 N bytes there).
        tm.tm_profile_enable(ctx, True)
        lb_ms = timed(lambda: step("lbfgs", n_lb, phase=False))
        d_ms, d_n = tm.tm_profile_query(ctx, 20)
        s_ms, s_n = tm.tm_profile_query(ctx, 21)
        tm.tm_profile_enable(ctx, False)
        m_lb = 5
        per_it = [(1 + (3 if it > 0 else 0) + 2 * min(it, m_lb)) * 8 * N * P for it in range(n_lb)]
        dbytes = float(np.mean(per_it))
        full = (1 + 3 + 2 * m_lb) * 8 * N * P
        d_avg = d_ms / max(d_n, 1)
        s_avg = s_ms / max(s_n, 1)
        gbs = dbytes / (d_avg * 1e-3) / 1e9
        tr_all = measured_traffic(P, N)
        tr_lb = tr_all.get("lbfgs_direction") if tr_all else None
        roofline_lbfgs = {
            "bound": "hbm", "kernel": "L-BFGS direction (k_dir_dots + k_dir_solve, compact form, m = 5; d formed in the line-search row kernel)",
            "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": tr_lb, "avg_launch_ms": round(d_avg, 5), "launches": d_n,
            "alg_bytes_per_launch": int(dbytes), "alg_bytes_full_history": int(full),
            "step_kernel": {"avg_launch_ms": round(s_avg, 5), "launches": s_n, "alg_bytes_per_launch": 4 * 8 * N * P,
                            "achieved_GBps": round(4 * 8 * N * P / (s_avg * 1e-3) / 1e9, 1)},
            "iteration_ms": round(lb_ms / n_lb, 4)}
    else:
        lb_ms = None
    la_ms = timed(lambda: step("lbfgs_amp", n_la, phase=False)) if n_la else None

    fid = fidelity(t).cpu().numpy()
    st = tm.decode_stats(raw)
    # phase correction quality: after diag(e^{j phi}) the rows share one offset w.r.t. the truth
    good = torch.from_numpy(fid >= 0.99).to(dev)
    off0 = torch.angle(torch.sum(torch.conj(t) * Tt, dim=1)).double()

    def spread(off):
        # circular standard deviation of the per-row offsets over rows retrieved to fidelity >= 0.99
        z = torch.exp(1j * off[good])
        return float(torch.sqrt(-2 * torch.log(torch.abs(z.mean()) + 1e-300)).item())

    phase_spread = spread(off0 - phi)
    phase_spread_before = spread(off0)

    # rooflines of the fused row kernels (one launch = one step over all P rows), timed live with HIP
    # events on the library's stream; the dominant one (largest total time in the timed region) is
    # `roofline`. Both are bound by FP32 vector arithmetic (the FFT work), so the primary figure is
    # against the vector peak; the HBM view carries the algorithmic bytes and the counter-measured traffic.
    flops_row = 2 * K * 5 * N * np.log2(N) + 30 * K * N  # 2K FFTs + pointwise per row-step
    wg_, rpw_, ept_ = tm.tm_config_info(n1, n2, tune["config"])
    cfg_note = (f" [launch configuration {tune['config']}: {wg_} threads, {rpw_} row(s) per workgroup, "
                f"{ept_} values per thread]")
    kernels = {
        "spectral": {"mode": sp_mode, "ms": sp_ms, "n": sp_n,
                     "name": "row_kernel<M_SPEC> (mask*FFT, truncated weights, IFFT, conj-mask sum, heavy-ball)"
                             if sp_mode == 5 else
                             "row_kernel<M_LANCZOS> (mask*FFT, truncated weights, IFFT, conj-mask sum, Lanczos step)",
                     # read I, v and the previous iterate, write the new v
                     "bytes": P * (K * N * 4 + 3 * N * 8)},
        "er": {"mode": er_mode, "ms": er_ms, "n": er_n,
               "name": "row_kernel<M_ER> (mask*FFT, amplitude projection, IFFT, conj-mask sum)" if solver == "er" else
                       "row_kernel<M_ERC> (per mask: mask*FFT, amplitude projection, IFFT, conj-mask)",
               # read I, t (and t_prev with momentum), write the new t
               "bytes": P * (K * N * 4 + (3 if beta > 0 else 2) * N * 8)},
    }
    # with two or more cyclic sweeps after the Lanczos start, the first sweep forms the Ritz vector itself:
    # it also reads the sp - 1 other basis rows and adds sp products per value (FP64 multiply-adds, 4 flops
    # per complex value); averaged over the solver's launches
    fused = solver == "er_cyclic" and args.start == "lanczos" and n_er >= 2
    er_extra_flops = (4 * sp * N) / n_er if fused else 0.0
    if fused:
        kernels["er"]["bytes"] += P * (sp - 1) * N * 8 / n_er
        kernels["er"]["name"] += "; the first sweep forms the Ritz vector from the Lanczos basis"
    # the first Lanczos step also forms the row sums of I and scales the seed to unit norm: one more read
    # of I, the seed written back and K N + 4 N additions per row; averaged over the start's launches
    sp_extra_flops = (K * N + 4 * N) / sp if sp_mode == 13 else 0.0
    if sp_mode == 13:
        kernels["spectral"]["bytes"] += P * (K * N * 4 + N * 8) / sp
        kernels["spectral"]["name"] += "; the first step also forms the row sums of I and the unit seed"
    extra_flops = {"er": er_extra_flops, "spectral": sp_extra_flops}
    for kv in kernels.values():
        kv["name"] += cfg_note
    traffic = measured_traffic(P, N, plan_tag(n1.bit_length() - 1, n2.bit_length() - 1, tune["config"]))
    roofs = {}
    for key, kv in kernels.items():
        avg = kv["ms"] / max(kv["n"], 1)
        tf = P * (flops_row + extra_flops[key]) / (avg * 1e-3) / 1e12
        gbs = kv["bytes"] / (avg * 1e-3) / 1e9
        tkey = {"er": "er_cyclic" if solver == "er_cyclic" else "er",
                "spectral": "lanczos" if sp_mode == 13 else "spectral"}[key]
        tr = traffic.get(tkey) if traffic else None
        roofs[key] = {
            "alu": {"bound": "alu", "kernel": kv["name"], "achieved": round(tf, 2), "peak": FP32_VALU_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(tf / FP32_VALU_PEAK_TFLOPS, 4),
                    "traffic": tr, "avg_launch_ms": round(avg, 5), "launches": kv["n"],
                    "alg_flops_per_launch": int(P * (flops_row + extra_flops[key])),
                    "alg_bytes_per_launch": int(kv["bytes"])},
            "hbm": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": tr},
        }
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    roofline = roofs[dom]["alu"]
    roofline_hbm = roofs[dom]["hbm"]
    other = [k for k in kernels if k != dom][0]
    er_avg_ms = er_ms / max(er_n, 1)

    out = {
        "metric": "TM rows/s to fidelity 0.99 at 2286x8192 (plain start)" if not args.small else
                  "TM rows/s to fidelity 0.99 at 512x1024 (plain start)",
        "value": round(P / (ms_step * 1e-3), 1),
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "P": P, "N": N, "grid": [n1, n2], "K": K,
                   "start": f"truncated spectral (tau {args.spectral_tau}), {sp} Lanczos steps" if args.start == "lanczos"
                            else f"truncated spectral (tau {args.spectral_tau}), {sp} heavy-ball steps "
                            f"(c {args.spectral_momentum}, interval [{args.spectral_lower}, c] lambda)",
                   "solver": (f"error reduction, Nesterov factor {beta}" if beta > 0 else "error reduction")
                             if solver == "er" else "cyclic error reduction (one mask projection at a time)",
                   "iters_to_0.99": n_er, "phase_iters": n_ph, "phase_evals": ph_ev, "phase_m": args.phase_m,
                   "phase_ftol": args.phase_ftol},
        "roofline": roofline,
        "roofline_hbm": roofline_hbm,
        "roofline_" + other: roofs[other]["alu"],
        "retrieval_ms": round(ret_ms, 3),
        "retrieval_rows_per_s": round(P / (ret_ms * 1e-3), 1),
        "phase_correction_ms": round(serial_ms - ret_ms, 3),
        "pipeline": {"enabled": bool(args.pipeline), "serial_ms_per_step": round(serial_ms, 3),
                     "serial_kernel_ms": serial_kernels,
                     "serial_roofline_frac": ({k: round(P * (flops_row + (er_extra_flops if k == "er_avg" else 0.0))
                                                         / (v * 1e-3) / 1e12 / FP32_VALU_PEAK_TFLOPS, 4)
                                               for k, v in serial_kernels.items()} if serial_kernels else None),
                     "serial_rows_per_s": round(P / (serial_ms * 1e-3), 1),
                     "note": "step i's phase solve on a second stream overlaps step i+1's retrieval; results "
                             "checked equal to the serial path" if args.pipeline else None},
        "lbfgs": {"iters_to_0.99": n_lb, "retrieval_ms": round(lb_ms, 3) if lb_ms else None},
        "roofline_lbfgs": roofline_lbfgs,
        "autotune": {"config": tune["config"], "shape_wg_rows_values": tm.tm_config_info(n1, n2, tune["config"]),
                     "candidates_us": {c: [v["lanczos_us"], v["er_cyclic_us"]]
                                       for c, v in tune.get("candidates", {}).items()}},
        "lbfgs_amplitude": {"iters_to_0.99": n_la, "retrieval_ms": round(la_ms, 3) if la_ms else None},
        "quality": {"mean_fidelity": round(float(fid.mean()), 6), "min_fidelity": round(float(fid.min()), 6),
                    "frac_rows_ge_0.99": round(float((fid >= 0.99).mean()), 4),
                    "spectral_start_fidelity": round(f_start, 4),
                    "rows_flagged_rho_gt_1e-2": int((st.flags.numpy() & 1).sum()),
                    "phase_spread_rad_before": round(phase_spread_before, 4),
                    "phase_spread_rad_after": round(phase_spread, 6),
                    "phase_spread_rows": int(good.sum().item())},
        "kernel_ms": {"er_avg": round(er_avg_ms, 5), "spectral_avg": round(sp_ms / max(sp_n, 1), 5),
                      "residual_f64_avg": round(rs_ms / max(rs_n, 1), 5)},
    }

    if not args.no_foci:
        out["foci"] = foci_variant(ctx, Tt, t, pixt, grid, P, N)
        out["foci_3d"] = foci3d_variant(ctx, Tt, t, phi, pixt, grid, (lam, ps, NA), P, N)
    if not args.no_dense and not args.small:
        out["dense_comparator"] = dense_variant(ctx, mk, It, t, n1, n2)
    if not args.no_learned:
        out["learned"] = learned_variant(args, ctx, mk, It, v0t, n1, n2, sp, n_er, fidelity, ret_ms, P)
    if not args.no_batch and not args.small:
        out["batch"] = batch_variant(ctx, args, pool)
    if not args.no_preprocess and not args.small:
        out["preprocess"] = preprocess_variant(ctx, args)
    if pool is not None:
        out["cpu_baseline"] = cpu_baseline(args, pool, masks, n1, n2, v0, I_np, T, theta, pix, nf, optics, Id_np,
                                           sp, n_er, beta, n_ph, P, solver, t.cpu().numpy(), phi.cpu().numpy(),
                                           ms_step)
        pool.shutdown()
    ctx.close()
    print(json.dumps(out), flush=True)


def learned_variant(args, ctx, mk, It, v0t, n1, n2, sp, n_er, fidelity, ret_ms, P):
    """Learned start on the same workload: the weighting network of the
    spectral start is trained on forward-model rows with this workload's masks
    (untimed); each form's (Lanczos steps, cyclic sweeps) is the cheapest
    that reaches mean fidelity 0.99 with at least 99 % of the rows at 0.99
    (untimed instrumented runs); then the learned form, with the per-row
    fallback to the plain start for rows whose FP64 residual stays above
    1e-2, is timed against the plain form."""
    import torch

    import paper_2302_13524_amd as tm
    from paper_2302_13524_amd import learned

    a = time.perf_counter()
    net, hist = learned.train_weights(ctx, mk, n1, n2, steps=args.train_steps, rows=128,
                                      power_steps=args.train_power_steps)
    learned.install_weights(ctx, net)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - a
    h = hist.cpu().numpy()

    def ok(start, k, s):
        t = v0t.clone()
        tm.tm_retrieve(ctx, mk, It, t, n1, n2, tm.retrieve_opts("er_cyclic", iters=s, start=start, spectral_iters=k,
                                                                 spectral_tau=args.spectral_tau), stats=False)
        f = fidelity(t)
        return f.mean().item() >= 0.99 and (f >= 0.99).double().mean().item() >= 0.99, f

    best = None
    for k in range(8, sp + 1):
        for s in range(1, 11):
            if best is not None and k + s >= best[0]:
                break
            good, f = ok("learned", k, s)
            if good:
                best = (k + s, k, s, float(f.mean().item()))
                break
    if best is None:
        return {"error": "the learned start did not reach the fidelity bar", "train_s": round(train_s, 2)}
    _, kl, sl, _ = best
    opts = tm.retrieve_opts("er_cyclic", iters=sl, start="learned", spectral_iters=kl, spectral_tau=args.spectral_tau)
    t0 = v0t.clone()
    tm.tm_retrieve(ctx, mk, It, t0, n1, n2, tm.retrieve_opts("er_cyclic", iters=0, start="learned",
                                                             spectral_iters=kl))
    f_start = float(fidelity(t0).mean().item())

    def run(rho):
        t = v0t.clone()
        if rho is None:
            raw = tm.tm_retrieve(ctx, mk, It, t, n1, n2, opts)
            return t, raw, 0
        raw, nf = tm.tm_retrieve_learned(ctx, mk, It, t, n1, n2, opts, rho_fallback=rho)
        return t, raw, nf

    def timed(rho, reps=5):
        run(rho)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            t, raw, nf = run(rho)
        torch.cuda.synchronize()
        return (time.perf_counter() - a) * 1e3 / reps, t, raw, nf

    rho_fb = args.learned_rho_fallback if args.learned_rho_fallback > 0 else None
    ms, t, raw, redone = timed(rho_fb)
    variants = {}
    for r in (None, 1e-1, 1e-2):
        if r == rho_fb:
            continue
        vms, vt, vraw, vnf = timed(r)
        vf = fidelity(vt)
        variants["no_fallback" if r is None else f"fallback_rho_{r:g}"] = {
            "retrieval_ms": round(vms, 3), "rows_redone": vnf, "final_mean_fidelity": round(float(vf.mean().item()), 6),
            "frac_rows_ge_0.99": round(float((vf >= 0.99).double().mean().item()), 4)}
    rho = tm.decode_stats(raw).rho.numpy()
    f = fidelity(t)
    return {"rows_per_s": round(P / (ms * 1e-3), 1), "retrieval_ms": round(ms, 3),
            "plain_retrieval_ms": round(ret_ms, 3), "gain": round(ret_ms / ms, 4),
            "lanczos_steps": kl, "sweeps": sl, "plain_lanczos_steps": sp, "plain_sweeps": n_er,
            "start_fidelity": round(f_start, 5), "rho_fallback": rho_fb, "rows_redone_from_fallback": redone,
            "final_rows_rho_gt_1e-2": int((rho > 1e-2).sum()),
            "final_mean_fidelity": round(float(f.mean().item()), 6),
            "frac_rows_ge_0.99": round(float((f >= 0.99).double().mean().item()), 4),
            "variants": variants,
            "train_steps": args.train_steps, "train_rows_per_step": 128, "train_power_steps": args.train_power_steps,
            "train_s": round(train_s, 2), "train_loss_first_last": [round(float(h[:10].mean()), 5),
                                                                    round(float(h[-10:].mean()), 5)]}


def foci_variant(ctx, Tt, t, pixt, grid, P, N):
    """Foci of the retrieved rows (Sec. 3 validation): the phase of each row's
    conjugate on the modulator, the true TM forms the image, PR = power in the
    7 x 7 window around the peak over the total. Also the true TM's own PR
    (the reference the paper takes from holography)."""
    import torch

    import paper_2302_13524_amd as tm

    pr, peak = tm.tm_foci_power_ratio(ctx, Tt, t, pixt, grid, grid, 3)
    pr_ref, _ = tm.tm_foci_power_ratio(ctx, Tt, Tt, pixt, grid, grid, 3)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        tm.tm_foci_power_ratio(ctx, Tt, t, pixt, grid, grid, 3)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    flops = 8.0 * P * P * N  # the complex GEMM
    on_target = float((peak == pixt).float().mean().item())
    return {"pr_mean": round(float(pr.mean().item()), 4), "pr_mean_true_tm": round(float(pr_ref.mean().item()), 4),
            "frac_peak_on_pixel": round(on_target, 4), "ms": round(ms, 3),
            "gemm_tflops": round(flops / (ms * 1e-3) / 1e12, 1), "window": 7}


def foci3d_variant(ctx, Tt, t, phi, pixt, grid, lam_ps_na, P, N, zs=(10.0, 20.0, 40.0)):
    """3-D foci (Sec. 4): the TM at a plane z for every pixel of the output
    grid (angular-spectrum propagation of each column), foci there from the
    retrieved rows with and without the phase-offset correction, images
    formed by the true TM propagated the same way. The correction is what
    makes the propagated estimate usable: without it every row carries its
    own unknown phase."""
    import torch

    import paper_2302_13524_amd as tm

    G = grid * grid
    allpix = torch.arange(G, dtype=torch.int32, device=pixt.device)
    tc = t * torch.exp(1j * phi).to(torch.complex64)[:, None]
    res = []
    prop_ms = None
    for z in zs:
        optics = (*lam_ps_na, z)
        Tz = tm.tm_propagate_tm(ctx, Tt, pixt, grid, grid, optics)
        tcz = tm.tm_propagate_tm(ctx, tc, pixt, grid, grid, optics)
        tuz = tm.tm_propagate_tm(ctx, t, pixt, grid, grid, optics)
        if prop_ms is None:
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(3):
                tm.tm_propagate_tm(ctx, tc, pixt, grid, grid, optics)
            e1.record()
            torch.cuda.synchronize()
            prop_ms = e0.elapsed_time(e1) / 3
        # foci aimed at the fiber-core pixels, images over the whole grid
        tgt = pixt.long()
        pr_c, pk_c = tm.tm_foci_power_ratio(ctx, Tz, tcz[tgt].contiguous(), allpix, grid, grid, 3)
        pr_u, _ = tm.tm_foci_power_ratio(ctx, Tz, tuz[tgt].contiguous(), allpix, grid, grid, 3)
        pr_t, pk_t = tm.tm_foci_power_ratio(ctx, Tz, Tz[tgt].contiguous(), allpix, grid, grid, 3)
        res.append({"z": z, "pr_mean_corrected": round(float(pr_c.mean().item()), 4),
                    "pr_mean_uncorrected": round(float(pr_u.mean().item()), 4),
                    "pr_mean_true_tm": round(float(pr_t.mean().item()), 4),
                    "frac_peak_on_target_corrected": round(float((pk_c == pixt).float().mean().item()), 4),
                    "frac_peak_on_target_true_tm": round(float((pk_t == pixt).float().mean().item()), 4)})
        del Tz, tcz, tuz
    return {"planes": res, "propagate_ms": round(prop_ms, 3), "grid": [grid, grid], "window": 7}


def dense_variant(ctx, mk, It, t, n1, n2):
    """Comparator without FFTs (Table time of the paper, on this GPU): one
    gradient evaluation of the intensity cost with a dense random-phase
    probing matrix Q [K N][N] (two complex FP32 GEMMs through rocBLAS, plus
    the pointwise step) against the fused FFT gradient kernel on the same rows."""
    import torch

    import paper_2302_13524_amd as tm

    dev = torch.device("cuda:0")
    K, N = mk.shape
    P = t.shape[0]
    g = torch.Generator(device=dev)
    g.manual_seed(91)
    Q = torch.polar(torch.ones((K * N, N), device=dev), 2 * np.pi * torch.rand((K * N, N), generator=g, device=dev))
    Q = Q.to(torch.complex64).contiguous()
    I2 = It.reshape(P, K * N).contiguous()

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    d_ms = timed(lambda: tm.tm_dense_gradient(ctx, Q, I2, t))
    f_ms = timed(lambda: tm.tm_gradient(ctx, mk, It, t, n1, n2), reps=10)
    flops = 2 * 8.0 * P * N * K * N
    del Q
    torch.cuda.empty_cache()
    return {"dense_gradient_ms": round(d_ms, 2), "fft_gradient_ms": round(f_ms, 4),
            "speedup_fft": round(d_ms / f_ms, 1), "dense_gemm_tflops": round(flops / (d_ms * 1e-3) / 1e12, 1),
            "M": K * N, "N": N, "P": P}


def preprocess_variant(ctx, args):
    """Preprocessing at the paper's camera layout: K N = 32768 images of
    128 x 128 uint16 counts (speckle inside a fiber disk of radius 54, dim
    background), half-sampled energy, 99.9 % fiber mask, per-pixel rows.
    The stack is synthesised on the GPU (seeded); each call is event-timed."""
    import torch

    import paper_2302_13524_amd as tm

    dev = torch.device("cuda:0")
    n_img, H, W, radius = 4 * 8192, 128, 128, 54.0
    g = torch.Generator(device=dev)
    g.manual_seed(77)
    y = torch.arange(H, device=dev, dtype=torch.float32)[:, None] - (H - 1) / 2
    x = torch.arange(W, device=dev, dtype=torch.float32)[None, :] - (W - 1) / 2
    inside = (y * y + x * x) <= radius * radius
    stack = torch.empty((n_img, H, W), dtype=torch.int16, device=dev)
    for i0 in range(0, n_img, 4096):  # in slabs, to bound the float temporaries
        u = torch.rand((min(4096, n_img - i0), H, W), generator=g, device=dev)
        v = torch.where(inside, torch.floor(-1000.0 * torch.log1p(-u)).clamp_(max=65535.0),
                        torch.floor(u * 1.05))  # background: 0, or 1 with probability 0.05
        stack[i0:i0 + v.shape[0]] = v.to(torch.int32).to(torch.int16)  # uint16 bits
        del u, v
    torch.cuda.synchronize()

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            r = fn()
        e1.record()
        torch.cuda.synchronize()
        return r, e0.elapsed_time(e1) / reps

    E, e_ms = timed(lambda: tm.tm_pre_energy(ctx, stack))
    pix, m_ms = timed(lambda: tm.tm_pre_fiber_mask(ctx, E, 0.999))
    rows, g_ms = timed(lambda: tm.tm_pre_gather(ctx, stack, pix))
    P = int(pix.numel())
    kept = n_img * (H // 2) * (W // 2) * 2  # bytes of the values used
    e_bytes, g_bytes = kept, P * n_img * (2 + 4)
    out = {"n_img": n_img, "image": [H, W], "P": P, "energy_ms": round(e_ms, 4), "mask_ms": round(m_ms, 4),
           "gather_ms": round(g_ms, 4), "total_ms": round(e_ms + m_ms + g_ms, 4),
           "energy_GBps": round(e_bytes / (e_ms * 1e-3) / 1e9, 1),
           "gather_GBps": round(g_bytes / (g_ms * 1e-3) / 1e9, 1),
           "energy_frac_hbm": round(e_bytes / (e_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "gather_frac_hbm": round(g_bytes / (g_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "alg_bytes": {"energy": e_bytes, "gather": g_bytes}}
    del stack, rows
    return out


def batch_variant(ctx, args, pool=None):
    """Twelve TMs of uneven (N, P) in one persistent launch per iteration under
    a captured HIP graph, BF16 intensities, digit order autotuned per grid.
    With the host workers (pool), the intensities come from the oracle's
    forward model and a seeded sample of rows of every TM is retrieved by the
    FP64 oracle from the same BF16-rounded values, so that each TM reports
    its fidelity against the oracle's rows."""
    import torch

    import paper_2302_13524_amd as tm
    import tm_synth

    dev = torch.device("cuda:0")
    shapes = [(32, 32, 512, 32), (64, 32, 900, 64), (64, 64, 1500, 64), (128, 64, 2286, 64)] * 3
    probs, truths = [], []
    a = time.perf_counter()
    for i, (n1, n2, P, grid) in enumerate(shapes):
        N = n1 * n2
        cid = 50 + i
        masks = torch.from_numpy(tm_synth.mask_phases(4, N, tm_synth.rng(cid, 0)).astype(np.complex64)).to(dev)
        pix = tm_synth.nearest_pixels(grid, P)
        T = torch.from_numpy(tm_synth.speckle_tm(N, grid, 0.22, pix, tm_synth.rng(cid, 1)).astype(np.complex64)).to(dev)
        if pool is not None:
            mk_np = masks.cpu().numpy()
            Ic = np.concatenate(list(pool.map(_oracle_intensities, [(mk_np.astype(np.complex128), n1, n2,
                                                                      T.cpu().numpy()[a0:b0])
                                                                     for a0, b0 in _cpu_chunks(P, pool.n_workers)])))
        else:
            Ic = tm.tm_forward(ctx, masks, T, n1, n2, intensity=True).cpu().numpy().astype(np.float64)
        I = tm_synth.poisson_counts(Ic, 1e4, tm_synth.rng(cid, 2))
        Ib = torch.from_numpy(I.astype(np.float32)).to(dev).to(torch.bfloat16)
        seed = torch.from_numpy(tm_synth.random_start(P, N, np.ones(P), tm_synth.rng(cid, 3)).astype(np.complex64)).to(dev)
        probs.append({"n1": n1, "n2": n2, "masks": masks, "I": Ib, "t": seed.clone(), "seed": seed,
                      "stats": torch.empty((P, tm.ROW_STATS_BYTES), dtype=torch.uint8, device=dev)})
        truths.append(T / torch.linalg.vector_norm(T, dim=1, keepdim=True))
    log(f"batch inputs {time.perf_counter() - a:.1f}s")
    tuned = {f"{n1}x{n2}": tm.autotune(ctx, n1, n2, 4, 512, bf16=True) for n1, n2, _, _ in shapes[:4]}
    iters, sp = args.batch_iters, args.batch_spectral_iters
    beta = args.er_momentum if args.solver == "er" else 0.0
    b = tm.Batch(ctx, probs, tm.retrieve_opts(args.solver, iters=iters, start=args.batch_start, spectral_iters=sp,
                                              bf16=True,
                                              spectral_tau=args.batch_spectral_tau,
                                              spectral_momentum=args.spectral_momentum,
                                              spectral_lower=args.spectral_lower,
                                              er_momentum=beta), use_graph=True)

    def run():
        for p in probs:
            p["t"].copy_(p["seed"])
        b.run()

    run()
    torch.cuda.synchronize()
    reps = 3
    ms = 0.0
    for _ in range(reps):
        for p in probs:
            p["t"].copy_(p["seed"])
        torch.cuda.synchronize()
        a = time.perf_counter()
        b.run()
        torch.cuda.synchronize()
        ms += (time.perf_counter() - a) * 1e3 / reps
    rows = sum(P for _, _, P, _ in shapes)
    per_tm = []
    jobs = []
    for i, (p, Tn) in enumerate(zip(probs, truths)):
        c = torch.sum(torch.conj(p["t"]) * Tn, dim=1)
        f = (c.abs() ** 2 / torch.sum(p["t"].abs() ** 2, dim=1)).double()
        per_tm.append({"grid": f"{p['n1']}x{p['n2']}", "P": p["t"].shape[0], "mean_fidelity": round(f.mean().item(), 5),
                       "rows_flagged": int((tm.decode_stats(p["stats"]).flags.numpy() & 1).sum())})
        if pool is not None:
            # a seeded sample of rows through the oracle's same pipeline, from the same BF16 values
            P = p["t"].shape[0]
            rows_s = np.sort(np.random.default_rng(900 + i).choice(P, 8, replace=False))
            Iv = p["I"].float().cpu().numpy()[rows_s].astype(np.float64)
            jobs.append((i, rows_s, pool.submit(_oracle_retrieve, (
                p["masks"].cpu().numpy().astype(np.complex128), p["n1"], p["n2"], Iv,
                p["seed"].cpu().numpy()[rows_s].astype(np.complex128), args.batch_start, sp, args.batch_spectral_tau,
                args.spectral_momentum, args.spectral_lower, args.solver, iters, beta))))
    for i, rows_s, fut in jobs:
        from oracle import retrieval as rt
        t_or, _ = fut.result()
        got = probs[i]["t"].cpu().numpy()[rows_s].astype(np.complex128)
        fo = rt.fidelity(got, t_or)
        per_tm[i]["sampled_rows"] = len(rows_s)
        per_tm[i]["gpu_vs_oracle_1_minus_fidelity_max"] = float(np.max(1 - fo))
    b.close()
    return {"rows_per_s": round(rows / (ms * 1e-3), 1), "ms": round(ms, 3), "rows": rows, "tms": len(shapes),
            "solver": args.solver, "start": args.batch_start, "iters": iters, "er_momentum": beta,
            "spectral_iters": sp,
            "spectral_tau": args.batch_spectral_tau, "dtype_I": "bf16", "variants": tuned, "per_tm": per_tm}


POOL_MAX = 16  # host worker processes (the CPU share of one GPU on the benchmark machines)


def cpu_pool():
    """Worker processes for the oracle legs, one BLAS thread each, started
    (spawned) before this process touches the GPU."""
    import concurrent.futures as cf
    import multiprocessing as mp
    n = max(1, min(POOL_MAX, len(os.sched_getaffinity(0))))
    keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in keep:
        os.environ[k] = "1"
    pool = cf.ProcessPoolExecutor(max_workers=n, mp_context=mp.get_context("spawn"))
    list(pool.map(_cpu_ready, range(n)))  # the workers exist (and have imported numpy) before the GPU is used
    for k, v in keep.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v
    pool.n_workers = n
    return pool


def _cpu_ready(_):
    return os.getpid()


def _cpu_chunks(P, n):
    step = max(1, -(-P // (4 * n)))
    return [(a, min(P, a + step)) for a in range(0, P, step)]


def _oracle_intensities(job):
    from oracle import operators as ops
    masks, n1, n2, T = job
    return ops.intensities(ops.FFTOp(masks, n1, n2), T.astype(np.complex128))


def _oracle_defocus(job):
    from oracle import defocus as df
    T, theta, pix, nf, optics = job
    lam, ps, NA, z = optics
    model = df.DefocusModel(T.astype(np.complex128), theta.astype(np.complex128), pix, nf, nf, lam, ps, NA, z)
    return model.images(np.zeros(T.shape[0]))


def _oracle_retrieve(job):
    from oracle import operators as ops
    from oracle import retrieval as rt
    masks, n1, n2, I, v0, start, sp, tau, mom, lower, solver, n_er, beta = job
    a = time.perf_counter()
    op = ops.FFTOp(masks, n1, n2)
    if start == "lanczos":
        t = rt.spectral_lanczos(op, I, v0, sp, tau=tau)
    else:
        t = rt.spectral_start(op, I, v0, sp, tau=tau, momentum=mom, lower=lower)
    t = rt.er_cyclic(masks, n1, n2, I, t, n_er) if solver == "er_cyclic" else rt.er_accelerated(op, I, t, n_er, beta)
    return t, time.perf_counter() - a


def _oracle_phase(job):
    from oracle import defocus as df
    t_est, theta, pix, nf, optics, Id, n_ph, m = job
    lam, ps, NA, z = optics
    a = time.perf_counter()
    model = df.DefocusModel(t_est, theta.astype(np.complex128), pix, nf, nf, lam, ps, NA, z)
    phi, _ = df.lbfgs_phase(model, Id, np.zeros(t_est.shape[0]), n_ph, m=m)
    return phi, time.perf_counter() - a


def oracle_inputs(pool, masks, T, n1, n2, theta, pix, nf, optics):
    """Clean intensities [P, K, N] and defocus images (FP64) by the oracle's
    forward models, in row chunks on the host workers."""
    P = T.shape[0]
    m = masks.astype(np.complex64).astype(np.complex128)  # the values the GPU receives
    chunks = _cpu_chunks(P, pool.n_workers)
    parts = pool.map(_oracle_intensities, [(m, n1, n2, T[a:b]) for a, b in chunks])
    Ic = np.concatenate(list(parts), axis=0)
    Idc = pool.submit(_oracle_defocus, (T, theta, pix, nf, optics)).result()
    return Ic, Idc


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, pool, masks, n1, n2, v0, I_np, T, theta, pix, nf, optics, Id_np, sp, n_er, beta, n_ph, P,
                 solver, t_gpu, phi_gpu, gpu_ms):
    """The FP64 oracle running the same path on the host's cores: the same
    spectral start and error-reduction sweeps over every row (row chunks on
    the worker processes, one thread each), then the phase-offset solve (one
    worker; it couples all pixels) from the oracle's own rows, with the same
    iteration counts and the same FP32 inputs as the GPU. Reports its
    throughput and how far the GPU's rows and offsets are from the oracle's."""
    from oracle import defocus as df
    from oracle import retrieval as rt

    m = masks.astype(np.complex64).astype(np.complex128)
    Iv = I_np.astype(np.float64)
    v = v0.astype(np.complex64).astype(np.complex128)
    chunks = _cpu_chunks(P, pool.n_workers)
    jobs = [(m, n1, n2, Iv[a:b], v[a:b], args.start, sp, args.spectral_tau, args.spectral_momentum,
             args.spectral_lower, solver, n_er, beta) for a, b in chunks]
    a0 = time.perf_counter()
    res = list(pool.map(_oracle_retrieve, jobs))
    ret_s = time.perf_counter() - a0
    t_or = np.concatenate([r[0] for r in res], axis=0)
    busy = sum(r[1] for r in res)
    a1 = time.perf_counter()
    phi_or, ph_s = pool.submit(_oracle_phase, (t_or, theta, pix, nf, optics, Id_np.astype(np.float64), n_ph,
                                               args.phase_m)).result()
    ph_wall = time.perf_counter() - a1
    total = ret_s + ph_wall
    fid_to_oracle = rt.fidelity(t_gpu.astype(np.complex128), t_or)
    fid_or = rt.fidelity(t_or, T.astype(np.complex128))
    fid_gpu = rt.fidelity(t_gpu.astype(np.complex128), T.astype(np.complex128))
    good = fid_or >= 0.99
    dphi = df.circular_offset_error(phi_gpu[good], phi_or[good]) if good.any() else np.zeros(1)
    return {"value": round(P / total, 3), "unit": "rows/s", "cores": pool.n_workers, "kind": "oracle",
            "sample": f"all {P} rows (no extrapolation): FP64 numpy FFT form of A, {sp} "
                      + ("Lanczos" if args.start == "lanczos" else "heavy-ball") + f" steps + {n_er} "
                      + (f"ER iterations (Nesterov factor {beta})" if solver == "er" else "cyclic ER sweeps")
                      + f" in {len(chunks)} row chunks over {pool.n_workers} worker processes ({ret_s:.1f} s wall, "
                      f"{busy:.1f} s of worker time), then the FP64 phase-offset L-BFGS over all pixels, "
                      f"{n_ph} iterations, memory {args.phase_m}, one worker ({ph_s:.1f} s); the same FP32 "
                      "intensities and defocus images as the GPU (oracle forward models, seeded Poisson noise)",
            "retrieval_s": round(ret_s, 3), "phase_s": round(ph_wall, 3),
            "cpu_model": cpu_model(), "host_cpus": len(os.sched_getaffinity(0)),
            "gpu_over_cpu": round(total * 1e3 / gpu_ms, 1),
            "oracle_mean_fidelity": round(float(fid_or.mean()), 6),
            "gpu_mean_fidelity": round(float(fid_gpu.mean()), 6),
            "mean_fidelity_diff": float(abs(fid_gpu.mean() - fid_or.mean())),
            "gpu_vs_oracle_1_minus_fidelity": {"max": float(np.max(1 - fid_to_oracle)),
                                               "mean": float(np.mean(1 - fid_to_oracle))},
            "gpu_vs_oracle_phase_rad": {"max": float(np.max(np.abs(dphi))), "rows": int(good.sum())}}


if __name__ == "__main__":
    main()
