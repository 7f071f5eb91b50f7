"""Python binding of libtm.so (include/tm.h): reference-less TM retrieval with
Fourier-structured probing on MI355X (gfx950).

Argument marshalling only: every step of the method runs in the library's
HIP kernels. Tensors are torch device tensors (contiguous; complex64 for
complex data, float32 or bfloat16 for intensities); the current torch
stream of the tensor's device is passed to the library. The names mirror
the C entry points. Importing works without a GPU; calling anything needs
the built library and a GPU, and fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtm.so")

TM_OK, TM_EINVAL, TM_EUNSUPPORTED, TM_EHIP, TM_ENOMEM = 0, -1, -2, -3, -4
TM_F32, TM_BF16 = 0, 1
TM_FIELD, TM_INTENSITY = 0, 1
TM_METHOD_ER, TM_METHOD_LBFGS, TM_METHOD_LBFGS_AMP, TM_METHOD_ER_CYCLIC = 0, 1, 2, 3
TM_START_GIVEN, TM_START_BACKPROP, TM_START_SPECTRAL, TM_START_LANCZOS, TM_START_LEARNED = 0, 1, 2, 3, 4
TM_WNET_FEATURES, TM_WTAB_MAX = 64, 4096

EXPORTED = (
    "tm_create", "tm_destroy", "tm_last_error", "tm_grid_supported", "tm_forward", "tm_adjoint",
    "tm_gradient", "tm_residual_f64", "tm_retrieve", "tm_phase_offset_correct", "tm_phase_objective",
    "tm_defocus_forward", "tm_profile_enable", "tm_profile_query",
    "tm_mlp_sync_bf16", "tm_mlp_start", "tm_mlp_gradients", "tm_mlp_train_step", "tm_gemm_bf16",
    "tm_batch_create", "tm_batch_run", "tm_batch_destroy", "tm_tune_time", "tm_set_variant",
    "tm_pre_energy", "tm_pre_fiber_mask", "tm_pre_gather", "tm_amp_gradient", "tm_foci_power_ratio",
    "tm_dense_gradient", "tm_propagate_tm", "tm_phase_set_band", "tm_phase_last_counts",
    "tm_retrieve_noalloc", "tm_wnet_table", "tm_wnet_pretrain_step", "tm_wtab_power_grad", "tm_wnet_train_step",
    "tm_set_weight_table", "tm_retrieve_learned", "tm_config_info", "tm_set_config", "tm_tune_config",
    "tm_cgemm_f32", "tm_phase_offset_correct_async",
)
TM_NOALLOC_MAX_ROWS = 32768
MODE_NAMES = {0: "forward_field", 1: "forward_intensity", 2: "adjoint", 3: "er", 4: "gradient", 5: "spectral",
              6: "line_sums", 7: "residual_f64", 8: "backprop", 9: "amp_gradient", 10: "amp_line_sums",
              11: "filter", 12: "er_cyclic", 13: "lanczos"}


class tm_dims(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("K", ctypes.c_int32), ("P", ctypes.c_int32)]


class tm_retrieve_opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("iters", ctypes.c_int32), ("lbfgs_m", ctypes.c_int32),
                ("I_dtype", ctypes.c_int32), ("start", ctypes.c_int32), ("spectral_iters", ctypes.c_int32),
                ("spectral_tau", ctypes.c_float), ("spectral_momentum", ctypes.c_float),
                ("er_momentum", ctypes.c_float), ("spectral_lower", ctypes.c_float)]


class tm_defocus_dims(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int32), ("N", ctypes.c_int32), ("Nd", ctypes.c_int32),
                ("nf1", ctypes.c_int32), ("nf2", ctypes.c_int32)]


class tm_optics(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("ps_field", ctypes.c_double), ("NA", ctypes.c_double),
                ("z", ctypes.c_double)]


class tm_phase_opts(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("m", ctypes.c_int32), ("ftol", ctypes.c_double)]


class tm_mlp_dims(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("hidden", ctypes.c_int32), ("n_out", ctypes.c_int32)]


_P3 = ctypes.c_void_p * 3


class tm_mlp_params(ctypes.Structure):
    _fields_ = [("W", _P3), ("Wh", _P3), ("b", _P3), ("mW", _P3), ("vW", _P3), ("mb", _P3), ("vb", _P3)]


class tm_problem(ctypes.Structure):
    _fields_ = [("d", tm_dims), ("masks", ctypes.c_void_p), ("I", ctypes.c_void_p), ("t", ctypes.c_void_p),
                ("stats", ctypes.c_void_p)]


ROW_STATS_BYTES = 24

_lib = None


class TMError(RuntimeError):
    pass


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libtm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise TMError(f"{path} not found: build it with paper_2302_13524_amd/build.py "
                      "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    vp, i32, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.tm_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.tm_destroy.argtypes = [vp]
    lib.tm_last_error.argtypes = [vp]
    lib.tm_last_error.restype = ctypes.c_char_p
    lib.tm_grid_supported.argtypes = [i32, i32]
    lib.tm_forward.argtypes = [vp, tm_dims, vp, vp, ctypes.c_int, ctypes.c_int, vp, vp]
    lib.tm_adjoint.argtypes = [vp, tm_dims, vp, vp, vp, vp]
    lib.tm_gradient.argtypes = [vp, tm_dims, vp, vp, ctypes.c_int, vp, vp, vp, vp]
    lib.tm_amp_gradient.argtypes = [vp, tm_dims, vp, vp, ctypes.c_int, vp, vp, vp, vp]
    lib.tm_residual_f64.argtypes = [vp, tm_dims, vp, vp, ctypes.c_int, vp, vp, vp]
    lib.tm_retrieve.argtypes = [vp, tm_dims, vp, vp, vp, ctypes.POINTER(tm_retrieve_opts), vp, vp]
    lib.tm_retrieve_noalloc.argtypes = [vp, tm_dims, vp, vp, vp, ctypes.POINTER(tm_retrieve_opts), vp, vp]
    f32 = ctypes.c_float
    lib.tm_wnet_table.argtypes = [vp, ctypes.POINTER(tm_mlp_dims), ctypes.POINTER(tm_mlp_params), i32, f32, vp, vp]
    lib.tm_wnet_pretrain_step.argtypes = [vp, ctypes.POINTER(tm_mlp_dims), ctypes.POINTER(tm_mlp_params), i32, f32,
                                          f32, f32, i32, vp, vp]
    lib.tm_wtab_power_grad.argtypes = [vp, tm_dims, vp, vp, i32, vp, vp, i32, vp, i32, f32, vp, vp, vp]
    lib.tm_wnet_train_step.argtypes = [vp, ctypes.POINTER(tm_mlp_dims), ctypes.POINTER(tm_mlp_params), tm_dims, vp,
                                       vp, i32, vp, vp, i32, i32, f32, f32, i32, vp, vp]
    lib.tm_set_weight_table.argtypes = [vp, vp, i32, f32, vp]
    lib.tm_retrieve_learned.argtypes = [vp, tm_dims, vp, vp, vp, ctypes.POINTER(tm_retrieve_opts), dp, vp,
                                        ctypes.POINTER(i32), vp]
    lib.tm_phase_offset_correct.argtypes = [vp, ctypes.POINTER(tm_defocus_dims), vp, vp, vp, vp,
                                            ctypes.POINTER(tm_optics), vp, ctypes.POINTER(tm_phase_opts),
                                            ctypes.POINTER(dp), vp]
    lib.tm_phase_offset_correct_async.argtypes = [vp, ctypes.POINTER(tm_defocus_dims), vp, vp, vp, vp,
                                                   ctypes.POINTER(tm_optics), vp, ctypes.POINTER(tm_phase_opts),
                                                   i32, vp, vp]
    lib.tm_phase_objective.argtypes = [vp, ctypes.POINTER(tm_defocus_dims), vp, vp, vp, vp,
                                       ctypes.POINTER(tm_optics), vp, vp, vp, vp]
    lib.tm_defocus_forward.argtypes = [vp, ctypes.POINTER(tm_defocus_dims), vp, vp, vp,
                                       ctypes.POINTER(tm_optics), vp, vp, vp]
    lib.tm_profile_enable.argtypes = [vp, ctypes.c_int]
    MD, MP = ctypes.POINTER(tm_mlp_dims), ctypes.POINTER(tm_mlp_params)
    lib.tm_mlp_sync_bf16.argtypes = [vp, MD, MP, vp]
    lib.tm_mlp_start.argtypes = [vp, MD, MP, i32, i32, vp, i32, vp, vp]
    lib.tm_mlp_gradients.argtypes = [vp, MD, MP, i32, i32, vp, vp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                     vp, vp]
    lib.tm_mlp_train_step.argtypes = [vp, MD, MP, i32, i32, vp, vp, i32, ctypes.c_float, i32, vp, vp]
    lib.tm_gemm_bf16.argtypes = [vp, i32, i32, i32, vp, i32, vp, i32, vp, vp]
    lib.tm_batch_create.argtypes = [vp, i32, ctypes.POINTER(tm_problem), ctypes.POINTER(tm_retrieve_opts), i32,
                                    ctypes.POINTER(vp)]
    lib.tm_batch_run.argtypes = [vp, vp]
    lib.tm_batch_destroy.argtypes = [vp]
    lib.tm_tune_time.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, ctypes.POINTER(dp)]
    lib.tm_set_variant.argtypes = [vp, i32, i32, i32]
    lib.tm_config_info.argtypes = [i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.tm_set_config.argtypes = [vp, i32, i32, i32]
    lib.tm_cgemm_f32.argtypes = [vp, i32, i32, i32, vp, ctypes.c_int64, vp, ctypes.c_int64, i32, vp, ctypes.c_int64,
                                 i32, vp]
    lib.tm_tune_config.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, ctypes.POINTER(dp)]
    lib.tm_phase_set_band.argtypes = [vp, i32]
    lib.tm_phase_last_counts.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.tm_profile_query.argtypes = [vp, ctypes.c_int, ctypes.POINTER(dp), ctypes.POINTER(ctypes.c_int64)]
    i64 = ctypes.c_int64
    lib.tm_pre_energy.argtypes = [vp, vp, i32, i64, i32, i32, vp, vp]
    lib.tm_pre_fiber_mask.argtypes = [vp, vp, i32, dp, vp, ctypes.POINTER(i32), vp]
    lib.tm_pre_gather.argtypes = [vp, vp, i32, i64, i32, i32, vp, i32, vp, i32, vp]
    lib.tm_foci_power_ratio.argtypes = [vp, i32, i32, i32, vp, vp, vp, i32, i32, i32, vp, vp, vp]
    lib.tm_dense_gradient.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp]
    lib.tm_propagate_tm.argtypes = [vp, i32, i32, vp, vp, i32, i32, ctypes.POINTER(tm_optics), vp, vp]
    _lib = lib
    return lib


def _ptr(x) -> int | None:
    if x is None:
        return None
    if not x.is_cuda:
        raise TMError("tensor must live on the GPU")
    if not x.is_contiguous():
        raise TMError("tensor must be contiguous")
    return x.data_ptr()


_C64 = (torch.complex64,)
_F32 = (torch.float32,)
_I32 = (torch.int32,)
_IDT = (torch.float32, torch.bfloat16, torch.int16, torch.uint16)


def _chk(x, name: str, shape, dtypes, dev=None) -> None:
    """Reject a tensor whose shape, dtype or device differs from what the C
    entry point will assume for its pointer (the library sees only the
    pointer and the sizes, so it cannot catch these itself)."""
    if not isinstance(x, torch.Tensor):
        raise TMError(f"{name}: expected a tensor, got {type(x).__name__}")
    if tuple(x.shape) != tuple(int(v) for v in shape):
        raise TMError(f"{name}: shape {tuple(x.shape)}, expected {tuple(int(v) for v in shape)}")
    if x.dtype not in dtypes:
        raise TMError(f"{name}: dtype {x.dtype}, expected one of {[str(d) for d in dtypes]}")
    if dev is not None and x.device != dev:
        raise TMError(f"{name}: on {x.device}, the other arguments are on {dev}")


def _grid(n1, n2, N) -> None:
    if int(n1) * int(n2) != int(N):
        raise TMError(f"grid {n1} x {n2} does not hold N = {N} modes")


def _masks(masks, n1, n2):
    if not isinstance(masks, torch.Tensor) or masks.dim() != 2:
        raise TMError("masks must be a [K, N] tensor")
    K, N = masks.shape
    _chk(masks, "masks", (K, N), _C64)
    _grid(n1, n2, N)
    return K, N


def _rows(t, name: str, N: int, dev) -> int:
    if not isinstance(t, torch.Tensor) or t.dim() != 2:
        raise TMError(f"{name} must be a [P, N] tensor")
    P = t.shape[0]
    _chk(t, name, (P, N), _C64, dev)
    return P


def _stream(dev: torch.device) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def _idtype(I: torch.Tensor) -> int:
    if I.dtype == torch.float32:
        return TM_F32
    if I.dtype in (torch.bfloat16, torch.int16, torch.uint16):
        return TM_BF16
    raise TMError(f"intensity dtype {I.dtype} (float32 or bfloat16)")


class Context:
    """A library context on one GPU (tm_create / tm_destroy)."""

    def __init__(self, device: int = 0):
        self.lib = load()
        self.device = device
        h = ctypes.c_void_p()
        rc = self.lib.tm_create(ctypes.byref(h), device)
        if rc != TM_OK:
            raise TMError(f"tm_create: {self.lib.tm_last_error(None).decode()} ({rc})")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.tm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc: int, what: str):
        if rc != TM_OK:
            raise TMError(f"{what}: {self.lib.tm_last_error(self.h).decode()} (code {rc})")

    def grid_supported(self, n1: int, n2: int) -> bool:
        return bool(self.lib.tm_grid_supported(n1, n2))


def _dims(n1, n2, K, P) -> tm_dims:
    return tm_dims(int(n1), int(n2), int(K), int(P))


def _rows_and_I(masks, I, t, n1, n2):
    """Checks of masks [K, N], rows t [P, N] and intensities I [P, K, N]."""
    K, N = _masks(masks, n1, n2)
    P = _rows(t, "t", N, masks.device)
    _chk(I, "I", (P, K, N), _IDT, masks.device)
    return K, N, P


def tm_forward(ctx: Context, masks, t, n1, n2, intensity: bool = False, bf16: bool = False, out=None):
    """y = A t ([P, K, N] complex64) or I = |A t|^2 ([P, K, N] float32 / bfloat16)."""
    K, N = _masks(masks, n1, n2)
    P = _rows(t, "t", N, masks.device)
    dt = torch.complex64 if not intensity else (torch.bfloat16 if bf16 else torch.float32)
    if out is None:
        out = torch.empty((P, K, N), dtype=dt, device=t.device)
    else:
        _chk(out, "out", (P, K, N), (dt,), t.device)
    rc = ctx.lib.tm_forward(ctx.h, _dims(n1, n2, K, P), _ptr(masks), _ptr(t),
                            TM_INTENSITY if intensity else TM_FIELD, TM_BF16 if bf16 else TM_F32,
                            _ptr(out), _stream(t.device))
    ctx.check(rc, "tm_forward")
    return out


def tm_adjoint(ctx: Context, masks, y, n1, n2, out=None):
    """x = A^H y, y [P, K, N] complex64 -> [P, N] complex64."""
    K, N = _masks(masks, n1, n2)
    if not isinstance(y, torch.Tensor) or y.dim() != 3:
        raise TMError("y must be a [P, K, N] tensor")
    P = y.shape[0]
    _chk(y, "y", (P, K, N), _C64, masks.device)
    if out is None:
        out = torch.empty((P, N), dtype=torch.complex64, device=y.device)
    else:
        _chk(out, "out", (P, N), _C64, y.device)
    rc = ctx.lib.tm_adjoint(ctx.h, _dims(n1, n2, K, P), _ptr(masks), _ptr(y), _ptr(out), _stream(y.device))
    ctx.check(rc, "tm_adjoint")
    return out


def tm_gradient(ctx: Context, masks, I, t, n1, n2):
    """Packed gradient -4 A^H((A t)(I - |A t|^2)) and f per row."""
    K, N, P = _rows_and_I(masks, I, t, n1, n2)
    g = torch.empty((P, N), dtype=torch.complex64, device=t.device)
    f = torch.empty((P,), dtype=torch.float32, device=t.device)
    rc = ctx.lib.tm_gradient(ctx.h, _dims(n1, n2, K, P), _ptr(masks), _ptr(I), _idtype(I), _ptr(t), _ptr(g),
                             _ptr(f), _stream(t.device))
    ctx.check(rc, "tm_gradient")
    return g, f


def tm_amp_gradient(ctx: Context, masks, I, t, n1, n2):
    """Packed gradient -2 A^H((sqrt(I) - |A t|)(A t)/|A t|) and the amplitude cost per row."""
    K, N, P = _rows_and_I(masks, I, t, n1, n2)
    g = torch.empty((P, N), dtype=torch.complex64, device=t.device)
    f = torch.empty((P,), dtype=torch.float32, device=t.device)
    rc = ctx.lib.tm_amp_gradient(ctx.h, _dims(n1, n2, K, P), _ptr(masks), _ptr(I), _idtype(I), _ptr(t), _ptr(g),
                                 _ptr(f), _stream(t.device))
    ctx.check(rc, "tm_amp_gradient")
    return g, f


def tm_residual_f64(ctx: Context, masks, I, t, n1, n2):
    """FP64 acceptance residual ||I - |A t|^2||^2 / ||I||^2 per row."""
    K, N, P = _rows_and_I(masks, I, t, n1, n2)
    rho = torch.empty((P,), dtype=torch.float64, device=t.device)
    rc = ctx.lib.tm_residual_f64(ctx.h, _dims(n1, n2, K, P), _ptr(masks), _ptr(I), _idtype(I), _ptr(t),
                                 _ptr(rho), _stream(t.device))
    ctx.check(rc, "tm_residual_f64")
    return rho


@dataclass
class RowStats:
    rho: torch.Tensor
    f: torch.Tensor
    amp_res: torch.Tensor
    iters: torch.Tensor
    flags: torch.Tensor


def decode_stats(raw: torch.Tensor) -> RowStats:
    b = raw.cpu()
    return RowStats(rho=b[:, 0:8].contiguous().view(torch.float64).reshape(-1),
                    f=b[:, 8:12].contiguous().view(torch.float32).reshape(-1),
                    amp_res=b[:, 12:16].contiguous().view(torch.float32).reshape(-1),
                    iters=b[:, 16:20].contiguous().view(torch.int32).reshape(-1),
                    flags=b[:, 20:24].contiguous().view(torch.int32).reshape(-1))


def retrieve_opts(method="er", iters=100, lbfgs_m=5, bf16=False, start="given", spectral_iters=30,
                  spectral_tau=3.0, spectral_momentum=0.98, er_momentum=0.0,
                  spectral_lower=None) -> tm_retrieve_opts:
    m = {"er": TM_METHOD_ER, "lbfgs": TM_METHOD_LBFGS, "lbfgs_amp": TM_METHOD_LBFGS_AMP,
         "er_cyclic": TM_METHOD_ER_CYCLIC}[method]
    s = {"given": TM_START_GIVEN, "backprop": TM_START_BACKPROP, "spectral": TM_START_SPECTRAL,
         "lanczos": TM_START_LANCZOS, "learned": TM_START_LEARNED}[start]
    return tm_retrieve_opts(m, int(iters), int(lbfgs_m), TM_BF16 if bf16 else TM_F32, s, int(spectral_iters),
                            float(spectral_tau), float(spectral_momentum), float(er_momentum),
                            float(-spectral_momentum if spectral_lower is None else spectral_lower))


def tm_retrieve(ctx: Context, masks, I, t, n1, n2, opts: tm_retrieve_opts | None = None, stats=True, **kw):
    """Retrieve every row in place in t ([P, N] complex64); returns the raw
    per-row stats tensor ([P, 24] uint8, see decode_stats) or None."""
    K, N, P = _rows_and_I(masks, I, t, n1, n2)
    if opts is None:
        opts = retrieve_opts(bf16=(I.dtype != torch.float32), **kw)
    if (opts.I_dtype == TM_F32) != (I.dtype == torch.float32):
        raise TMError(f"I dtype {I.dtype} does not match opts.I_dtype {opts.I_dtype}")
    raw = torch.empty((P, ROW_STATS_BYTES), dtype=torch.uint8, device=t.device) if stats else None
    rc = ctx.lib.tm_retrieve(ctx.h, _dims(n1, n2, K, P), _ptr(masks), _ptr(I), _ptr(t), ctypes.byref(opts),
                             _ptr(raw), _stream(t.device))
    ctx.check(rc, "tm_retrieve")
    return raw


def tm_retrieve_noalloc(ctx: Context, masks, I, t, n1, n2, opts: tm_retrieve_opts, stats=None):
    """tm_retrieve for error reduction from a given or back-propagation start,
    with no device allocation in the library (its sums use a static device
    array shared by every call on the device). stats: None or a caller-owned
    [P, 24] uint8 device tensor."""
    K, N, P = _rows_and_I(masks, I, t, n1, n2)
    if (opts.I_dtype == TM_F32) != (I.dtype == torch.float32):
        raise TMError(f"I dtype {I.dtype} does not match opts.I_dtype {opts.I_dtype}")
    if stats is not None:
        _chk(stats, "stats", (P, ROW_STATS_BYTES), (torch.uint8,), t.device)
    rc = ctx.lib.tm_retrieve_noalloc(ctx.h, _dims(n1, n2, K, P), _ptr(masks), _ptr(I), _ptr(t), ctypes.byref(opts),
                                     _ptr(stats), _stream(t.device))
    ctx.check(rc, "tm_retrieve_noalloc")
    return stats


def _ddims(P, N, Nd, nf1, nf2):
    return tm_defocus_dims(int(P), int(N), int(Nd), int(nf1), int(nf2))


def _defocus_args(pix, tm_rows, theta, nf1, nf2, I_d=None, phi=None):
    """Checks of the defocus-model arguments: tm_rows [P, N], pix [P] int32,
    theta [Nd, N] complex64, I_d [Nd, 2 nf1, 2 nf2] float32, phi [P] float64."""
    if not isinstance(tm_rows, torch.Tensor) or tm_rows.dim() != 2:
        raise TMError("tm rows must be a [P, N] tensor")
    P, N = tm_rows.shape
    dev = tm_rows.device
    _chk(tm_rows, "tm rows", (P, N), _C64)
    _chk(pix, "pix", (P,), _I32, dev)
    if not isinstance(theta, torch.Tensor) or theta.dim() != 2:
        raise TMError("theta must be a [Nd, N] tensor")
    Nd = theta.shape[0]
    _chk(theta, "theta", (Nd, N), _C64, dev)
    if I_d is not None:
        _chk(I_d, "I_d", (Nd, 2 * int(nf1), 2 * int(nf2)), _F32, dev)
    if phi is not None:
        _chk(phi, "phi", (P,), (torch.float64,), dev)
    return P, N, Nd


def tm_phase_objective(ctx: Context, pix, tm_est, theta, I_d, optics, phi, nf1, nf2):
    """g(phi) and dg/dphi of the defocus problem (FP64)."""
    P, N, Nd = _defocus_args(pix, tm_est, theta, nf1, nf2, I_d, phi)
    g = torch.empty((1,), dtype=torch.float64, device=tm_est.device)
    grad = torch.empty((P,), dtype=torch.float64, device=tm_est.device)
    dd = _ddims(P, N, Nd, nf1, nf2)
    op = tm_optics(*[float(v) for v in optics])
    rc = ctx.lib.tm_phase_objective(ctx.h, ctypes.byref(dd), _ptr(pix), _ptr(tm_est), _ptr(theta), _ptr(I_d),
                                    ctypes.byref(op), _ptr(phi), _ptr(g), _ptr(grad), _stream(tm_est.device))
    ctx.check(rc, "tm_phase_objective")
    return g, grad


def tm_phase_offset_correct(ctx: Context, pix, tm_est, theta, I_d, optics, phi, nf1, nf2, iters=100, m=5, ftol=0.0):
    """Solve the per-row phase offsets in place in phi ([P] float64); returns g.
    Stops early after an accepted iteration that lowers g by at most ftol * g."""
    P, N, Nd = _defocus_args(pix, tm_est, theta, nf1, nf2, I_d, phi)
    dd = _ddims(P, N, Nd, nf1, nf2)
    op = tm_optics(*[float(v) for v in optics])
    po = tm_phase_opts(int(iters), int(m), float(ftol))
    g = ctypes.c_double(0.0)
    rc = ctx.lib.tm_phase_offset_correct(ctx.h, ctypes.byref(dd), _ptr(pix), _ptr(tm_est), _ptr(theta),
                                         _ptr(I_d), ctypes.byref(op), _ptr(phi), ctypes.byref(po),
                                         ctypes.byref(g), _stream(tm_est.device))
    ctx.check(rc, "tm_phase_offset_correct")
    return g.value


def tm_phase_offset_correct_async(ctx: Context, pix, tm_est, theta, I_d, optics, phi, nf1, nf2, rec, evals,
                                  iters=100, m=5, ftol=0.0):
    """Stream-ordered phase solve: queues `evals` device L-BFGS iterations and returns at once; the
    record (g, iterations, evaluations, ended, pixel check, rows) lands in rec ([>= 7] float64, device)."""
    P, N, Nd = _defocus_args(pix, tm_est, theta, nf1, nf2, I_d, phi)
    if not (isinstance(rec, torch.Tensor) and rec.dtype == torch.float64 and rec.is_contiguous()
            and rec.numel() >= 7 and rec.device == tm_est.device):
        raise TMError("rec must be a contiguous float64 tensor of >= 7 values on the device of tm_est")
    dd = _ddims(P, N, Nd, nf1, nf2)
    op = tm_optics(*[float(v) for v in optics])
    po = tm_phase_opts(int(iters), int(m), float(ftol))
    rc = ctx.lib.tm_phase_offset_correct_async(ctx.h, ctypes.byref(dd), _ptr(pix), _ptr(tm_est), _ptr(theta),
                                               _ptr(I_d), ctypes.byref(op), _ptr(phi), ctypes.byref(po),
                                               int(evals), _ptr(rec), _stream(tm_est.device))
    ctx.check(rc, "tm_phase_offset_correct_async")


TM_U16 = 2


def _stack_dtype(stack) -> int:
    if stack.dim() != 3:
        raise TMError("stack must be [n_img, H, W]")
    if stack.dtype in (torch.int16, torch.uint16):  # camera counts (int16 tensors carry the uint16 bits)
        return TM_U16
    if stack.dtype == torch.float32:
        return TM_F32
    raise TMError(f"stack dtype {stack.dtype}: uint16 camera counts or float32")


def tm_pre_energy(ctx: Context, stack):
    """Summed intensity of every half-sampled pixel, [(H/2)*(W/2)] float64."""
    n, H, W = stack.shape
    out = torch.empty(((H // 2) * (W // 2),), dtype=torch.float64, device=stack.device)
    rc = ctx.lib.tm_pre_energy(ctx.h, _ptr(stack), _stack_dtype(stack), int(n), int(H), int(W), _ptr(out),
                               _stream(stack.device))
    ctx.check(rc, "tm_pre_energy")
    return out


def tm_pre_fiber_mask(ctx: Context, energy, frac=0.999):
    """Ascending raster indices of the brightest-first pixel set holding frac of the total, int32 [P]."""
    if not isinstance(energy, torch.Tensor) or energy.dim() != 1:
        raise TMError("energy must be a 1-D tensor")
    _chk(energy, "energy", energy.shape, (torch.float64,))
    npix = energy.numel()
    pix = torch.empty((npix,), dtype=torch.int32, device=energy.device)
    P = ctypes.c_int32(0)
    rc = ctx.lib.tm_pre_fiber_mask(ctx.h, _ptr(energy), int(npix), float(frac), _ptr(pix), ctypes.byref(P),
                                   _stream(energy.device))
    ctx.check(rc, "tm_pre_fiber_mask")
    return pix[:P.value].clone()


def tm_pre_gather(ctx: Context, stack, pix, bf16=False):
    """Per-pixel rows [P, n_img]: out[p][i] = stack[i][2y][2x] for pix[p] = y*(W/2) + x."""
    _stack_dtype(stack)
    n, H, W = stack.shape
    if not isinstance(pix, torch.Tensor) or pix.dim() != 1:
        raise TMError("pix must be a 1-D tensor")
    _chk(pix, "pix", pix.shape, _I32, stack.device)
    P = pix.numel()
    out = torch.empty((P, n), dtype=torch.bfloat16 if bf16 else torch.float32, device=stack.device)
    rc = ctx.lib.tm_pre_gather(ctx.h, _ptr(stack), _stack_dtype(stack), int(n), int(H), int(W),
                               _ptr(pix) if P else None, int(P), _ptr(out) if P else None,
                               TM_BF16 if bf16 else TM_F32, _stream(stack.device))
    ctx.check(rc, "tm_pre_gather")
    return out


def tm_propagate_tm(ctx: Context, tm_rows, pix, g1, g2, optics):
    """TM at the plane optics[3] (= z) for every pixel of the g1 x g2 grid: [g1*g2, N] complex64."""
    if not isinstance(tm_rows, torch.Tensor) or tm_rows.dim() != 2:
        raise TMError("tm_rows must be a [P, N] tensor")
    P, N = tm_rows.shape
    _chk(tm_rows, "tm_rows", (P, N), _C64)
    _chk(pix, "pix", (P,), _I32, tm_rows.device)
    out = torch.empty((g1 * g2, N), dtype=torch.complex64, device=tm_rows.device)
    op = tm_optics(*[float(v) for v in optics])
    rc = ctx.lib.tm_propagate_tm(ctx.h, int(P), int(N), _ptr(tm_rows), _ptr(pix), int(g1), int(g2),
                                 ctypes.byref(op), _ptr(out), _stream(tm_rows.device))
    ctx.check(rc, "tm_propagate_tm")
    return out


def tm_dense_gradient(ctx: Context, Q, I, t):
    """Gradient -4 Q^H((Q t)(I - |Q t|^2)) and f per row for a dense probing matrix Q [M, N]."""
    if not isinstance(Q, torch.Tensor) or Q.dim() != 2:
        raise TMError("Q must be an [M, N] tensor")
    M, N = Q.shape
    _chk(Q, "Q", (M, N), _C64)
    P = _rows(t, "t", N, Q.device)
    _chk(I, "I", (P, M), _F32, Q.device)
    g = torch.empty((P, N), dtype=torch.complex64, device=t.device)
    f = torch.empty((P,), dtype=torch.float32, device=t.device)
    rc = ctx.lib.tm_dense_gradient(ctx.h, int(M), int(N), int(P), _ptr(Q), _ptr(I), _ptr(t), _ptr(g), _ptr(f),
                                   _stream(t.device))
    ctx.check(rc, "tm_dense_gradient")
    return g, f


def tm_foci_power_ratio(ctx: Context, tm_true, tm_est, pix, g1, g2, w=3):
    """Power ratio [Pf] float32 and peak raster index [Pf] int32 of the conjugate-phase focus of every
    row of tm_est [Pf, N], with images over the rows of tm_true [G, N] at the pixels pix [G]."""
    if not isinstance(tm_true, torch.Tensor) or tm_true.dim() != 2:
        raise TMError("tm_true must be a [G, N] tensor")
    G, N = tm_true.shape
    _chk(tm_true, "tm_true", (G, N), _C64)
    Pf = _rows(tm_est, "tm_est", N, tm_true.device)
    _chk(pix, "pix", (G,), _I32, tm_true.device)
    pr = torch.empty((Pf,), dtype=torch.float32, device=tm_true.device)
    peak = torch.empty((Pf,), dtype=torch.int32, device=tm_true.device)
    rc = ctx.lib.tm_foci_power_ratio(ctx.h, int(Pf), int(G), int(N), _ptr(tm_true), _ptr(pix), _ptr(tm_est),
                                     int(g1), int(g2), int(w), _ptr(pr), _ptr(peak), _stream(tm_true.device))
    ctx.check(rc, "tm_foci_power_ratio")
    return pr, peak


def tm_defocus_forward(ctx: Context, pix, tm_rows, theta, optics, phi, nf1, nf2):
    """Defocus images |A_n e^{j phi}|^2, [Nd, 2nf1, 2nf2] float32."""
    P, N, Nd = _defocus_args(pix, tm_rows, theta, nf1, nf2, None, phi)
    out = torch.empty((Nd, 2 * nf1, 2 * nf2), dtype=torch.float32, device=tm_rows.device)
    dd = _ddims(P, N, Nd, nf1, nf2)
    op = tm_optics(*[float(v) for v in optics])
    rc = ctx.lib.tm_defocus_forward(ctx.h, ctypes.byref(dd), _ptr(pix), _ptr(tm_rows), _ptr(theta),
                                    ctypes.byref(op), _ptr(phi), _ptr(out), _stream(tm_rows.device))
    ctx.check(rc, "tm_defocus_forward")
    return out


def tm_profile_enable(ctx: Context, enable: bool = True):
    ctx.check(ctx.lib.tm_profile_enable(ctx.h, 1 if enable else 0), "tm_profile_enable")


def tm_profile_query(ctx: Context, mode: int):
    """(total milliseconds, launches) of the fused row kernel `mode` since enabling."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    ctx.check(ctx.lib.tm_profile_query(ctx.h, int(mode), ctypes.byref(ms), ctypes.byref(n)), "tm_profile_query")
    return ms.value, n.value


class MLP:
    """Learned-start network parameters on the GPU (FP32 masters, BF16 copies,
    Adam moments); shapes W[l]: [fan_in][fan_out]."""

    def __init__(self, n_in: int, hidden: int, n_out: int, device="cuda:0", weights=None, seed: int = 0):
        self.dims = tm_mlp_dims(n_in, hidden, n_out)
        shapes = [(n_in, hidden), (hidden, hidden), (hidden, n_out)]
        if weights is None:
            g = torch.Generator().manual_seed(seed)
            weights = []
            for fi, fo in shapes:
                weights.append((torch.randn((fi, fo), generator=g) / fi ** 0.5, torch.zeros(fo)))
        self.W = [torch.as_tensor(w, dtype=torch.float32).contiguous().to(device) for w, _ in weights]
        self.b = [torch.as_tensor(b, dtype=torch.float32).contiguous().to(device) for _, b in weights]
        self.Wh = [torch.empty(w.shape, dtype=torch.bfloat16, device=device) for w in self.W]
        self.mW = [torch.zeros_like(w) for w in self.W]
        self.vW = [torch.zeros_like(w) for w in self.W]
        self.mb = [torch.zeros_like(b) for b in self.b]
        self.vb = [torch.zeros_like(b) for b in self.b]
        self.step = 0
        P3 = lambda xs: _P3(*[x.data_ptr() for x in xs])
        self.p = tm_mlp_params(P3(self.W), P3(self.Wh), P3(self.b), P3(self.mW), P3(self.vW), P3(self.mb),
                               P3(self.vb))

    def sync(self, ctx: Context):
        ctx.check(ctx.lib.tm_mlp_sync_bf16(ctx.h, ctypes.byref(self.dims), ctypes.byref(self.p),
                                           _stream(self.W[0].device)), "tm_mlp_sync_bf16")


def _mlp_io(net: MLP, K: int, N: int) -> None:
    if net.dims.n_in != K * N or net.dims.n_out != 2 * N:
        raise TMError(f"network {net.dims.n_in} -> {net.dims.n_out} does not map K N = {K * N} "
                      f"intensities to 2 N = {2 * N} values")


def _mlp_batch(net: MLP, I, t, K: int, N: int) -> int:
    if not isinstance(I, torch.Tensor) or I.dim() != 3:
        raise TMError("I must be a [B, K, N] tensor")
    B = I.shape[0]
    dev = net.W[0].device
    _chk(I, "I", (B, K, N), _F32, dev)
    _chk(t, "t", (B, N), _C64, dev)
    _mlp_io(net, K, N)
    return B


def tm_mlp_start(ctx: Context, net: MLP, I, K: int, N: int):
    """Learned start rows [P, N] complex64 from intensities [P, K, N] float32."""
    if not isinstance(I, torch.Tensor) or I.dim() != 3:
        raise TMError("I must be a [P, K, N] tensor")
    P = I.shape[0]
    _chk(I, "I", (P, K, N), _F32, net.W[0].device)
    _mlp_io(net, K, N)
    t0 = torch.empty((P, N), dtype=torch.complex64, device=I.device)
    rc = ctx.lib.tm_mlp_start(ctx.h, ctypes.byref(net.dims), ctypes.byref(net.p), K, N, _ptr(I), P, _ptr(t0),
                              _stream(I.device))
    ctx.check(rc, "tm_mlp_start")
    return t0


def tm_mlp_gradients(ctx: Context, net: MLP, I, t, K: int, N: int):
    """(dW list, db list, per-row loss) of the mean loss over the batch."""
    B = _mlp_batch(net, I, t, K, N)
    dW = [torch.empty_like(w) for w in net.W]
    db = [torch.empty_like(b) for b in net.b]
    loss = torch.empty((B,), dtype=torch.float32, device=I.device)
    pw = (ctypes.c_void_p * 3)(*[x.data_ptr() for x in dW])
    pb = (ctypes.c_void_p * 3)(*[x.data_ptr() for x in db])
    rc = ctx.lib.tm_mlp_gradients(ctx.h, ctypes.byref(net.dims), ctypes.byref(net.p), K, N, _ptr(I), _ptr(t), B,
                                  pw, pb, _ptr(loss), _stream(I.device))
    ctx.check(rc, "tm_mlp_gradients")
    return dW, db, loss


def tm_mlp_train_step(ctx: Context, net: MLP, I, t, K: int, N: int, lr: float, loss=None):
    B = _mlp_batch(net, I, t, K, N)
    if loss is not None:
        _chk(loss, "loss", (B,), _F32, I.device)
    net.step += 1
    rc = ctx.lib.tm_mlp_train_step(ctx.h, ctypes.byref(net.dims), ctypes.byref(net.p), K, N, _ptr(I), _ptr(t), B,
                                   float(lr), net.step, _ptr(loss), _stream(I.device))
    ctx.check(rc, "tm_mlp_train_step")


def tm_gemm_bf16(ctx: Context, A, B, ta=False, tb=False):
    """C = op(A) op(B) in FP32 from BF16 A, B."""
    if not isinstance(A, torch.Tensor) or not isinstance(B, torch.Tensor) or A.dim() != 2 or B.dim() != 2:
        raise TMError("A and B must be 2-D tensors")
    M = A.shape[1] if ta else A.shape[0]
    K = A.shape[0] if ta else A.shape[1]
    N = B.shape[0] if tb else B.shape[1]
    _chk(A, "A", A.shape, (torch.bfloat16,))
    _chk(B, "B", (N, K) if tb else (K, N), (torch.bfloat16,), A.device)
    C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    rc = ctx.lib.tm_gemm_bf16(ctx.h, M, N, K, _ptr(A), int(ta), _ptr(B), int(tb), _ptr(C), _stream(A.device))
    ctx.check(rc, "tm_gemm_bf16")
    return C


class Batch:
    """A planned retrieval of several problems of uneven size (tm_batch_*).
    problems: list of dicts with masks [K, N], I [P, K, N], t [P, N] (in/out),
    n1, n2 and optionally stats ([P, 24] uint8 device tensor)."""

    def __init__(self, ctx: Context, problems, opts: tm_retrieve_opts, use_graph: bool = True):
        self.ctx = ctx
        self.problems = problems  # keeps the tensors alive
        arr = (tm_problem * len(problems))()
        for i, p in enumerate(problems):
            K, N = _masks(p["masks"], p["n1"], p["n2"])
            P = _rows(p["t"], "t", N, p["masks"].device)
            _chk(p["I"], "I", (P, K, N), (torch.float32,) if opts.I_dtype == TM_F32 else _IDT[1:],
                 p["masks"].device)
            if p.get("stats") is not None:
                _chk(p["stats"], "stats", (P, ROW_STATS_BYTES), (torch.uint8,), p["masks"].device)
            arr[i] = tm_problem(_dims(p["n1"], p["n2"], K, p["t"].shape[0]), _ptr(p["masks"]), _ptr(p["I"]),
                                _ptr(p["t"]), _ptr(p.get("stats")))
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.tm_batch_create(ctx.h, len(problems), arr, ctypes.byref(opts), int(use_graph),
                                          ctypes.byref(h)), "tm_batch_create")
        self.h = h

    def run(self, stream=None):
        dev = self.problems[0]["t"].device
        self.ctx.check(self.ctx.lib.tm_batch_run(self.h, stream if stream is not None else _stream(dev)),
                       "tm_batch_run")

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.tm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tm_tune_time(ctx: Context, n1, n2, K, P, variant, bf16=False, reps=5) -> float:
    us = ctypes.c_double(0.0)
    ctx.check(ctx.lib.tm_tune_time(ctx.h, n1, n2, K, P, TM_BF16 if bf16 else TM_F32, variant, reps,
                                   ctypes.byref(us)), "tm_tune_time")
    return us.value


def tm_phase_set_band(ctx: Context, enable: bool):
    """Pupil-band (pruned) evaluation of the defocus model when the pupil's box is small (default on)."""
    ctx.check(ctx.lib.tm_phase_set_band(ctx.h, 1 if enable else 0), "tm_phase_set_band")


def tm_phase_last_counts(ctx: Context):
    """(accepted iterations, objective evaluations) of the context's last tm_phase_offset_correct."""
    it, ev = ctypes.c_int32(0), ctypes.c_int32(0)
    ctx.check(ctx.lib.tm_phase_last_counts(ctx.h, ctypes.byref(it), ctypes.byref(ev)), "tm_phase_last_counts")
    return it.value, ev.value


def tm_set_variant(ctx: Context, n1, n2, variant):
    ctx.check(ctx.lib.tm_set_variant(ctx.h, n1, n2, variant), "tm_set_variant")


def tm_cgemm_f32(ctx: Context, A, B, trans_b=False, conj_c=False):
    """C = A op(B) (complex64 on the device, matrix cores): A [M, K]; B [N, K]
    with trans_b, else [K, N]; conj(C) with conj_c."""
    if not isinstance(A, torch.Tensor) or not isinstance(B, torch.Tensor) or A.dim() != 2 or B.dim() != 2:
        raise TMError("A and B must be 2-D tensors")
    M, K = A.shape
    N = B.shape[0] if trans_b else B.shape[1]
    _chk(A, "A", (M, K), _C64)
    _chk(B, "B", (N, K) if trans_b else (K, N), _C64, A.device)
    C = torch.empty((M, N), dtype=torch.complex64, device=A.device)
    ctx.check(ctx.lib.tm_cgemm_f32(ctx.h, M, N, K, _ptr(A), K, _ptr(B), B.shape[1], int(bool(trans_b)), _ptr(C), N,
                                   int(bool(conj_c)), _stream(A.device)), "tm_cgemm_f32")
    return C


def tm_config_info(n1, n2, cfg):
    """(threads per workgroup, rows per workgroup, values per thread) of launch
    configuration cfg (0..7) for the grid, or None if it is not compiled."""
    if not isinstance(cfg, int) or isinstance(cfg, bool):
        raise TMError("cfg must be an int")
    wg, rpw, ept = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    ok = load().tm_config_info(int(n1), int(n2), int(cfg), ctypes.byref(wg), ctypes.byref(rpw), ctypes.byref(ept))
    return (wg.value, rpw.value, ept.value) if ok else None


def tm_set_config(ctx: Context, n1, n2, cfg):
    ctx.check(ctx.lib.tm_set_config(ctx.h, n1, n2, cfg), "tm_set_config")


def tm_tune_config(ctx: Context, n1, n2, K, P, cfg, bf16=False, reps=5):
    """(Lanczos-step us, cyclic ER-step us) of configuration cfg on synthetic data."""
    us = (ctypes.c_double * 2)()
    ctx.check(ctx.lib.tm_tune_config(ctx.h, n1, n2, K, P, TM_BF16 if bf16 else TM_F32, cfg, reps, us),
              "tm_tune_config")
    return us[0], us[1]


def autotune(ctx: Context, n1: int, n2: int, K: int, P: int, bf16: bool = False, cache: str | None = None,
             reps: int = 5, space: str = "digits") -> dict:
    """Choose the launch configuration of an n1 x n2 grid, apply it to the
    context and record it in the JSON cache `cache` (keyed by architecture,
    grid, K, intensity type and search space); a cached entry is applied
    without timing.

    space="digits": the two FFT digit orders, timed on the error-reduction
    kernel over P rows (what the uneven batch takes).
    space="full": every configuration compiled for the grid (digit order,
    eight or sixteen values per thread, one or two times the rows per
    workgroup, hence the waves per SIMD), each timed on the Lanczos step and
    the cyclic ER step over P rows; the one with the least sum is applied."""
    import json
    if space not in ("digits", "full"):
        raise TMError(f"space {space!r} (digits or full)")
    key = f"gfx950:{n1}x{n2}:K{K}:{'bf16' if bf16 else 'f32'}" + (":full" if space == "full" else "")
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            table = json.load(fh)
    if key in table:
        entry = table[key]
    elif space == "digits":
        times = [tm_tune_time(ctx, n1, n2, K, P, v, bf16, reps) for v in (0, 1)]
        entry = {"variant": int(times[1] < times[0]), "us": times, "rows": P}
    else:
        # two rounds over the candidates, each keeping its faster round, so that
        # the clock's ramp during the first launches favours none of them
        cand = {}
        for rnd in range(2):
            for cfg in range(8):
                shape = tm_config_info(n1, n2, cfg)
                if shape is None:
                    continue
                lz, er = tm_tune_config(ctx, n1, n2, K, P, cfg, bf16, reps)
                old = cand.get(str(cfg))
                if old is None or lz + er < old["lanczos_us"] + old["er_cyclic_us"]:
                    cand[str(cfg)] = {"lanczos_us": round(lz, 2), "er_cyclic_us": round(er, 2), "wg": shape[0],
                                      "rows_per_wg": shape[1], "values_per_thread": shape[2]}
        best = min(cand, key=lambda k: cand[k]["lanczos_us"] + cand[k]["er_cyclic_us"])
        entry = {"config": int(best), "variant": int(best) & 1, "candidates": cand, "rows": P}
    if cache and key not in table:
        table[key] = entry
        with open(cache, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
    if "config" in entry:
        tm_set_config(ctx, n1, n2, entry["config"])
    else:
        tm_set_variant(ctx, n1, n2, entry["variant"])
    return entry


# ---------------------------------------------------------------- learned weighting of the spectral start

def weight_net(hidden: int = 256, device="cuda:0", seed: int = 0) -> MLP:
    """The network that proposes the spectral start's weights T(x):
    TM_WNET_FEATURES features of x -> hidden -> hidden -> 1 (tm_wnet_*)."""
    return MLP(TM_WNET_FEATURES, hidden, 1, device=device, seed=seed)


def _wnet_check(net: MLP):
    if net.dims.n_in != TM_WNET_FEATURES or net.dims.n_out != 1:
        raise TMError(f"weight network must map {TM_WNET_FEATURES} features to 1 output")


def tm_wnet_table(ctx: Context, net: MLP, nt: int = 256, xmax: float = 16.0):
    """The network's weight table [nt, 2] float32: (T(x_b), T(x_{b+1}) - T(x_b))."""
    _wnet_check(net)
    tab = torch.empty((int(nt), 2), dtype=torch.float32, device=net.W[0].device)
    ctx.check(ctx.lib.tm_wnet_table(ctx.h, ctypes.byref(net.dims), ctypes.byref(net.p), int(nt), float(xmax),
                                    _ptr(tab), _stream(tab.device)), "tm_wnet_table")
    return tab


def tm_wnet_pretrain_step(ctx: Context, net: MLP, nt: int, xmax: float, tau: float, lr: float, loss=None):
    _wnet_check(net)
    if loss is not None:
        _chk(loss, "loss", (1,), _F32, net.W[0].device)
    net.step += 1
    ctx.check(ctx.lib.tm_wnet_pretrain_step(ctx.h, ctypes.byref(net.dims), ctypes.byref(net.p), int(nt), float(xmax),
                                            float(tau), float(lr), net.step, _ptr(loss),
                                            _stream(net.W[0].device)), "tm_wnet_pretrain_step")


def _wtab_rows(masks, I, t, v0, n1, n2):
    K, N, P = _rows_and_I(masks, I, t, n1, n2)
    _chk(v0, "v0", (P, N), _C64, masks.device)
    return K, N, P


def tm_wtab_power_grad(ctx: Context, masks, I, t, v0, n1, n2, tab, steps: int, xmax: float = 16.0):
    """(loss, d loss / d table values [nt]) of `steps` power steps with the table's weights."""
    K, N, P = _wtab_rows(masks, I, t, v0, n1, n2)
    if not isinstance(tab, torch.Tensor) or tab.dim() != 2:
        raise TMError("tab must be an [nt, 2] tensor")
    nt = tab.shape[0]
    _chk(tab, "tab", (nt, 2), _F32, masks.device)
    dtab = torch.empty((nt,), dtype=torch.float32, device=masks.device)
    loss = torch.empty((1,), dtype=torch.float32, device=masks.device)
    ctx.check(ctx.lib.tm_wtab_power_grad(ctx.h, _dims(n1, n2, K, P), _ptr(masks), _ptr(I), _idtype(I), _ptr(t),
                                         _ptr(v0), int(steps), _ptr(tab), int(nt), float(xmax), _ptr(dtab),
                                         _ptr(loss), _stream(masks.device)), "tm_wtab_power_grad")
    return loss, dtab


def tm_wnet_train_step(ctx: Context, net: MLP, masks, I, t, v0, n1, n2, steps: int, nt: int = 256,
                       xmax: float = 16.0, lr: float = 1e-3, loss=None):
    _wnet_check(net)
    K, N, P = _wtab_rows(masks, I, t, v0, n1, n2)
    if loss is not None:
        _chk(loss, "loss", (1,), _F32, masks.device)
    net.step += 1
    ctx.check(ctx.lib.tm_wnet_train_step(ctx.h, ctypes.byref(net.dims), ctypes.byref(net.p), _dims(n1, n2, K, P),
                                         _ptr(masks), _ptr(I), _idtype(I), _ptr(t), _ptr(v0), int(steps), int(nt),
                                         float(xmax), float(lr), net.step, _ptr(loss), _stream(masks.device)),
              "tm_wnet_train_step")


def tm_set_weight_table(ctx: Context, tab, xmax: float = 16.0):
    if not isinstance(tab, torch.Tensor) or tab.dim() != 2:
        raise TMError("tab must be an [nt, 2] tensor")
    _chk(tab, "tab", (tab.shape[0], 2), _F32)
    ctx.check(ctx.lib.tm_set_weight_table(ctx.h, _ptr(tab), int(tab.shape[0]), float(xmax), _stream(tab.device)),
              "tm_set_weight_table")


def tm_retrieve_learned(ctx: Context, masks, I, t, n1, n2, opts: tm_retrieve_opts, rho_fallback: float = 1e-2,
                        stats=True):
    """Learned-start retrieval in place in t with the plain start as per-row
    fallback; returns (raw stats [P, 24] uint8 or None, rows redone)."""
    K, N, P = _rows_and_I(masks, I, t, n1, n2)
    if opts.start != TM_START_LEARNED:
        raise TMError("opts.start must be 'learned'")
    if (opts.I_dtype == TM_F32) != (I.dtype == torch.float32):
        raise TMError(f"I dtype {I.dtype} does not match opts.I_dtype {opts.I_dtype}")
    raw = torch.empty((P, ROW_STATS_BYTES), dtype=torch.uint8, device=t.device) if stats else None
    nf = ctypes.c_int32(0)
    ctx.check(ctx.lib.tm_retrieve_learned(ctx.h, _dims(n1, n2, K, P), _ptr(masks), _ptr(I), _ptr(t),
                                          ctypes.byref(opts), float(rho_fallback), _ptr(raw), ctypes.byref(nf),
                                          _stream(t.device)), "tm_retrieve_learned")
    return raw, nf.value
