"""Singular value shrinkage by Chebyshev polynomial approximation on MI355X.

Thin ctypes binding over ``libcpasvt.so`` (C ABI in ``include/cpasvt.h``):
argument marshalling only.  Every step of the shrinkage runs in the library's
HIP kernels; torch supplies device memory and the current stream.  If the
library has not been built the calls raise ``RuntimeError`` -- there is no CPU
fallback.

Typical use::

    import torch, paper_1705_07112_amd as cpa
    X = torch.randn(1024, 1024, device="cuda")
    Y = cpa.shrink_dense(X, cpa.soft(10.0), cpa.Opts(K=30))
"""
from __future__ import annotations

import atexit
import ctypes
import os
import re
import weakref
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcpasvt.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "cpasvt.h")

SOFT, HARD, WEIGHTED_CONST, WEIGHTED_FN = 0, 1, 2, 3
BOUND_POWER, BOUND_GIVEN, BOUND_FROBENIUS, BOUND_LEARNED, BOUND_LANCZOS = 0, 1, 2, 3, 4
PREC_FP32, PREC_BF16X3, PREC_FP64 = 0, 1, 2
OK, ERR_ARG, ERR_SHAPE, ERR_ALLOC, ERR_HIP, ERR_NONFINITE, ERR_BOUND, ERR_UNSUPPORTED, ERR_IO = range(9)


class CpaShrinkage(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("tau", ctypes.c_double),
                ("w_c", ctypes.c_double), ("w_sigma", ctypes.c_double), ("w_eps", ctypes.c_double)]


class CpaOpts(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("bound", ctypes.c_int32), ("Lambda", ctypes.c_double),
                ("power_iters", ctypes.c_int32), ("warm_start", ctypes.c_int32),
                ("power_tol", ctypes.c_double), ("margin", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("check", ctypes.c_int32), ("precision", ctypes.c_int32), ("growth_tol", ctypes.c_double),
                ("eval", ctypes.c_int32), ("side", ctypes.c_int32), ("damping", ctypes.c_int32),
                ("lanczos_steps", ctypes.c_int32), ("model", ctypes.c_void_p), ("coeffs", ctypes.c_void_p)]


class CpaInfo(ctypes.Structure):
    _fields_ = [("Lambda", ctypes.c_double), ("mu", ctypes.c_double), ("resid", ctypes.c_double),
                ("fro_gram", ctypes.c_double), ("max_growth", ctypes.c_double),
                ("power_iters_done", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("side", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class CpaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_string(status)}: {message}")
        self.status = status


THRESHOLD_KEEP, THRESHOLD_ABSOLUTE = 0, 1


class CpaSparsify(ctypes.Structure):
    _fields_ = [("transform", ctypes.c_int32), ("threshold", ctypes.c_int32), ("keep", ctypes.c_int64),
                ("eps", ctypes.c_double)]


TRANSFORM_IDENTITY, TRANSFORM_BLOCK_DCT8, TRANSFORM_HAAR1, TRANSFORM_HAAR1_LOWPASS, TRANSFORM_DCT = 0, 1, 2, 3, 4
_TRANSFORMS = {"identity": TRANSFORM_IDENTITY, "block_dct8": TRANSFORM_BLOCK_DCT8, "haar1": TRANSFORM_HAAR1,
               "haar1_lowpass": TRANSFORM_HAAR1_LOWPASS, "dct": TRANSFORM_DCT}


class CpaBatchedTuning(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32), ("pair", ctypes.c_int32), ("order", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("best_us", ctypes.c_double), ("default_us", ctypes.c_double)]


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_SIGS = {
    "cpa_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]),
    "cpa_destroy": (ctypes.c_int, [_P]),
    "cpa_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "cpa_last_error": (ctypes.c_char_p, []),
    "cpa_default_opts": (None, [ctypes.POINTER(CpaOpts)]),
    "cpa_damping_factors": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P]),
    "cpa_chebyshev_coeffs": (ctypes.c_int, [ctypes.POINTER(CpaShrinkage), ctypes.c_double, ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_double)]),
    "cpa_design_coeffs": (ctypes.c_int, [ctypes.POINTER(CpaShrinkage), ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "cpa_spectral_bound": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, _P, _I64, ctypes.POINTER(CpaOpts),
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(CpaInfo)]),
    "cpa_shrink_dense": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, _P, _I64, _P, _I64,
                                        ctypes.POINTER(CpaShrinkage), ctypes.POINTER(CpaOpts),
                                        ctypes.POINTER(CpaInfo)]),
    "cpa_shrink_dense_noalloc": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, _P, _I64, _P, _I64,
                                                ctypes.POINTER(CpaShrinkage), ctypes.POINTER(CpaOpts),
                                                ctypes.POINTER(CpaInfo)]),
    "cpa_shrink_dense_f64": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, _P, _I64, _P, _I64,
                                        ctypes.POINTER(CpaShrinkage), ctypes.POINTER(CpaOpts),
                                        ctypes.POINTER(CpaInfo)]),
    "cpa_rpca_state_floats": (ctypes.c_int64, [ctypes.c_int, ctypes.c_int]),
    "cpa_predictor_save": (ctypes.c_int, [_P, _P, _P, ctypes.c_char_p]),
    "cpa_predictor_load": (ctypes.c_int, [_P, _P, ctypes.c_char_p, _P]),
    "cpa_rpca_admm": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, _P, _P, _P, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_double, ctypes.POINTER(CpaOpts), _P,
                                     ctypes.POINTER(ctypes.c_int)]),
    "cpa_inpaint_state_floats": (ctypes.c_int64, [ctypes.c_int, ctypes.c_int]),
    "cpa_inpaint_init": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, _P, _P]),
    "cpa_inpaint_iterate": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, _P, _P, _P, _P, ctypes.c_int,
                                           ctypes.c_double, ctypes.c_double, ctypes.POINTER(CpaOpts), _P]),
    "cpa_keep_schedule": (ctypes.c_int, [ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         ctypes.POINTER(ctypes.c_int64)]),
    "cpa_inpaint_iterate_scheduled": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, _P, _P, _P, _P,
                                                     ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                     ctypes.POINTER(CpaOpts), ctypes.c_int32, ctypes.c_double,
                                                     ctypes.c_double, ctypes.c_double, _P, _P]),
    "cpa_timing_enable": (ctypes.c_int, [_P, ctypes.c_int]),
    "cpa_peak_mfma": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]),
    "cpa_workspace_bytes": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(CpaOpts),
                                           ctypes.POINTER(ctypes.c_size_t)]),
    "cpa_timing_read": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]),
    "cpa_rpca_init": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, _P]),
    "cpa_shrink_csr": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _P, _P, _P, _P, _I64,
                                      ctypes.POINTER(CpaShrinkage), ctypes.POINTER(CpaOpts), ctypes.POINTER(CpaInfo)]),
    "cpa_svt_complete": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _P, _P, _P, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int, _P, _I64, ctypes.POINTER(CpaOpts), _P,
                                        ctypes.POINTER(ctypes.c_double), _P, _P, _P]),
    "cpa_shrink_batched": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, _P, _P, _P, _P, _P, ctypes.POINTER(CpaShrinkage),
                                          ctypes.POINTER(CpaOpts), _P, _P, _P]),
    "cpa_batched_features": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, _P, _P, _P, _P, _P]),
    "cpa_shrink_dense_sparsified": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, _P, _I64, _P, _I64,
                                                   ctypes.POINTER(CpaShrinkage), ctypes.POINTER(CpaOpts),
                                                   ctypes.POINTER(CpaSparsify), ctypes.POINTER(CpaInfo),
                                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "cpa_batched_plan_create": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, _P, _P, _P, _P, _P,
                                               ctypes.POINTER(CpaShrinkage), ctypes.POINTER(CpaOpts), _P, _P, _P,
                                               ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "cpa_batched_plan_execute": (ctypes.c_int, [_P, _P]),
    "cpa_batched_plan_tuning": (ctypes.c_int, [_P, ctypes.POINTER(CpaBatchedTuning)]),
    "cpa_batched_plan_destroy": (ctypes.c_int, [_P]),
    "cpa_shrink_batched_predicted": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, _P, _P, _P, _P, _P,
                                                    ctypes.POINTER(CpaShrinkage), ctypes.POINTER(CpaOpts), _P,
                                                    ctypes.c_int32, _P, _P, _P]),
    "cpa_predictor_forward": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P, _P]),
    "cpa_predictor_grad": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P, ctypes.POINTER(ctypes.c_float), _P, _P,
                                          _P]),
    "cpa_predictor_train": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P, ctypes.POINTER(ctypes.c_float),
                                           ctypes.c_int32, ctypes.c_int32, ctypes.c_float, _P, _P,
                                           ctypes.POINTER(ctypes.c_int64), _P]),
    "cpa_rpca_iterate": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, _P, _P, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_double, ctypes.POINTER(CpaOpts), _P]),
}


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run `python -m paper_1705_07112_amd.build`)")
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def declared_symbols() -> list[str]:
    """Function names declared in include/cpasvt.h."""
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cpa_[a-z0-9_]+)\s*\(", text)))


def status_string(s: int) -> str:
    return lib().cpa_status_string(int(s)).decode()


def _check(status: int):
    if status != 0:
        raise CpaError(status, lib().cpa_last_error().decode())


# ---- parameter helpers ------------------------------------------------------

def soft(tau: float) -> CpaShrinkage:
    return CpaShrinkage(SOFT, 0, float(tau), 0.0, 0.0, 1.0)


def hard(tau: float) -> CpaShrinkage:
    return CpaShrinkage(HARD, 0, float(tau), 0.0, 0.0, 1.0)


def weighted_const(w_over_rho: float) -> CpaShrinkage:
    return CpaShrinkage(WEIGHTED_CONST, 0, float(w_over_rho), 0.0, 0.0, 1.0)


def weighted_fn(w_c: float, w_sigma: float, w_eps: float = 1e-6) -> CpaShrinkage:
    return CpaShrinkage(WEIGHTED_FN, 0, 0.0, float(w_c), float(w_sigma), float(w_eps))


@dataclass
class Opts:
    K: int = 16
    bound: str = "power"          # "power" | "given" | "frobenius" | "learned" (needs model) | "lanczos"
    Lambda: float | None = None
    power_iters: int = 100
    warm_start: bool = False
    power_tol: float = 1e-7
    margin: float = 0.01
    seed: int = 0
    check: bool = False
    growth_tol: float = 1e-3
    precision: str = "fp32"      # "fp32" | "bf16x3" | "fp64" (FP64 inputs only)
    eval: str = "auto"           # "auto" | "recurrence" | "polynomial"
    side: str = "auto"           # "auto" | "right" (Gram X^T X) | "left" (Gram X X^T)
    damping: str = "none"        # "none" | "jackson" | "lanczos" (coefficient damping; not in the paper)
    lanczos_steps: int = 0        # bound "lanczos": steps (1..32; 0: the library's default, 12)
    model: object = None          # bound "learned": the predictor model (float32 CUDA tensor)
    coeffs: object = None         # caller-given coefficients (float64 CUDA tensor of K entries; bound "given")

    def to_c(self) -> CpaOpts:
        o = CpaOpts()
        lib().cpa_default_opts(ctypes.byref(o))
        o.K = int(self.K)
        bound = self.bound
        if self.Lambda is not None and bound == "power":
            bound = "given"
        o.bound = {"power": BOUND_POWER, "given": BOUND_GIVEN, "frobenius": BOUND_FROBENIUS,
                   "learned": BOUND_LEARNED, "lanczos": BOUND_LANCZOS}[bound]
        if self.model is not None:
            if self.model.dtype.itemsize != 4 or not self.model.is_cuda or not self.model.is_contiguous() \
                    or self.model.numel() != PRED_MODEL_FLOATS:
                raise ValueError("model must be a contiguous float32 CUDA tensor of %d entries" % PRED_MODEL_FLOATS)
            o.model = self.model.data_ptr()
        if self.coeffs is not None:
            if self.coeffs.dtype.itemsize != 8 or not self.coeffs.is_cuda or not self.coeffs.is_contiguous() \
                    or not self.coeffs.is_floating_point() or self.coeffs.numel() != int(self.K):
                raise ValueError("coeffs must be a contiguous float64 CUDA tensor of K entries")
            o.coeffs = self.coeffs.data_ptr()
        o.Lambda = float(self.Lambda or 0.0)
        o.power_iters = int(self.power_iters)
        o.warm_start = int(bool(self.warm_start))
        o.power_tol = float(self.power_tol)
        o.margin = float(self.margin)
        o.seed = int(self.seed)
        o.check = int(bool(self.check))
        o.precision = {"fp32": PREC_FP32, "bf16x3": PREC_BF16X3, "fp64": PREC_FP64}[self.precision]
        o.growth_tol = float(self.growth_tol)
        o.eval = {"auto": 0, "recurrence": 1, "polynomial": 2}[self.eval]
        o.side = {"auto": 0, "right": 1, "left": 2}[self.side]
        o.damping = {"none": 0, "jackson": 1, "lanczos": 2}[self.damping]
        o.lanczos_steps = int(self.lanczos_steps)
        return o


# ---- device plumbing -----------------------------------------------------------

_contexts: dict[int, int] = {}
_plans = weakref.WeakSet()       # open BatchedPlan objects


def context(device: int = 0) -> int:
    if device not in _contexts:
        h = ctypes.c_void_p()
        _check(lib().cpa_create(ctypes.byref(h), int(device)))
        _contexts[device] = h.value
    return _contexts[device]


def release() -> None:
    """Destroys every open batched plan and every context (their graphs, streams,
    events and device buffers).  Runs at interpreter exit, before the HIP runtime
    is torn down, so nothing the library owns is left for the runtime's own exit
    handlers; a later call creates a fresh context."""
    for p in list(_plans):
        try:
            p.close()
        except Exception:
            pass
    while _contexts:
        _, h = _contexts.popitem()
        lib().cpa_destroy(ctypes.c_void_p(h))


atexit.register(release)


def _stream(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _mat(t, name, dtypes=("float32",)):
    import torch
    ok = tuple(getattr(torch, d) for d in dtypes)
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype not in ok or t.dim() != 2:
        raise TypeError(f"{name} must be a 2-D {' or '.join(dtypes)} CUDA tensor")
    if t.shape[0] > 0 and t.shape[1] > 0:
        if t.stride(1) != 1 and t.shape[1] > 1:
            raise ValueError(f"{name} must have unit column stride (row-major)")
        if t.shape[0] > 1 and t.stride(0) < t.shape[1]:
            raise ValueError(f"{name} has rows that overlap (row stride {t.stride(0)} < {t.shape[1]} columns)")
    return t.shape[0], t.shape[1], max(t.stride(0), t.shape[1])


def chebyshev_coeffs(shrink: CpaShrinkage, Lambda: float, K: int) -> np.ndarray:
    """FP64 coefficients from the library's host routine."""
    out = (ctypes.c_double * int(K))()
    _check(lib().cpa_chebyshev_coeffs(ctypes.byref(shrink), float(Lambda), int(K), out))
    return np.array(out[:], dtype=np.float64)


DESIGNS = {"chebyshev": 0, "lsq": 1, "minimax": 2}


def design_coeffs(shrink: CpaShrinkage, Lambda: float, K: int, design: str, n: int = 0):
    """(coefficients, largest error on the design's points) of another polynomial design
    (cpa_design_coeffs), in the convention Opts.coeffs takes."""
    out = (ctypes.c_double * int(K))()
    err = ctypes.c_double()
    _check(lib().cpa_design_coeffs(ctypes.byref(shrink), float(Lambda), int(K), DESIGNS[design], int(n), out,
                                   ctypes.byref(err)))
    return np.array(out[:], dtype=np.float64), float(err.value)


def damping_factors(K: int, kind: str = "jackson"):
    """The coefficient damping factors g_0..g_{K-1} (cpa_damping_factors) as a list."""
    out = (ctypes.c_double * int(K))()
    _check(lib().cpa_damping_factors(int(K), {"none": 0, "jackson": 1, "lanczos": 2}[kind], out))
    return list(out)


SCHEDULE_E_L = 0.03
SCHEDULE_E_M = 6e-4


def keep_schedule(E_t: float, d: int, E_l: float = SCHEDULE_E_L, E_m: float = SCHEDULE_E_M) -> int:
    """The keep count of eq. (recommendation_epsilon) for E_t on a d x d transformed
    Gram (cpa_keep_schedule)."""
    k = ctypes.c_int64(0)
    _check(lib().cpa_keep_schedule(float(E_t), int(d), float(E_l), float(E_m), ctypes.byref(k)))
    return int(k.value)


def shrink_dense(X, shrink: CpaShrinkage, opts: Opts, out=None, info: bool = False):
    """Y = hat G(X) (Algorithm 1 with T = Id).  float32 X: cpa_shrink_dense;
    float64 X: cpa_shrink_dense_f64 (FP64 arithmetic).  Returns Y, or (Y, info dict)."""
    import torch
    m, n, ldx = _mat(X, "X", ("float32", "float64"))
    if out is None:
        out = torch.empty((m, n), device=X.device, dtype=X.dtype)
    _, _, ldy = _mat(out, "out", ("float32", "float64"))
    if tuple(out.shape) != (m, n) or out.dtype != X.dtype:
        raise ValueError("out has the wrong shape or dtype")
    ci = CpaInfo()
    co = opts.to_c()
    fn = lib().cpa_shrink_dense_f64 if X.dtype == torch.float64 else lib().cpa_shrink_dense
    _check(fn(ctypes.c_void_p(context(X.device.index or 0)), _stream(X), m, n, ctypes.c_void_p(X.data_ptr()), ldx,
              ctypes.c_void_p(out.data_ptr()), ldy, ctypes.byref(shrink), ctypes.byref(co),
              ctypes.byref(ci) if info else None))
    return (out, ci.as_dict()) if info else out


def shrink_dense_noalloc(X, shrink: CpaShrinkage, opts: Opts, out, info: bool = False):
    """cpa_shrink_dense_noalloc: the FP32 shrink with its workspace in the library's
    static scratch (the caller passes the output).  Returns out, or (out, info dict)."""
    m, n, ldx = _mat(X, "X")
    _, _, ldy = _mat(out, "out")
    if tuple(out.shape) != (m, n) or out.device != X.device:
        raise ValueError("out has the wrong shape or device")
    ci = CpaInfo()
    co = opts.to_c()
    _check(lib().cpa_shrink_dense_noalloc(ctypes.c_void_p(context(X.device.index or 0)), _stream(X), m, n,
                                          ctypes.c_void_p(X.data_ptr()), ldx, ctypes.c_void_p(out.data_ptr()), ldy,
                                          ctypes.byref(shrink), ctypes.byref(co), ctypes.byref(ci) if info else None))
    return (out, ci.as_dict()) if info else out


def spectral_bound(X, opts: Opts):
    """(Lambda, info dict) for the Gram of X, computed on the device."""
    m, n, ldx = _mat(X, "X")
    lam = ctypes.c_double()
    ci = CpaInfo()
    co = opts.to_c()
    _check(lib().cpa_spectral_bound(ctypes.c_void_p(context(X.device.index or 0)), _stream(X), m, n,
                                    ctypes.c_void_p(X.data_ptr()), ldx, ctypes.byref(co), ctypes.byref(lam),
                                    ctypes.byref(ci)))
    return lam.value, ci.as_dict()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def shrink_dense_sparsified(X, shrink: CpaShrinkage, opts: Opts, keep: int | None = None,
                            transform: str = "block_dct8", out=None, info: bool = False, eps: float | None = None):
    """Algorithm 1 with a transform and truncation (see cpa_shrink_dense_sparsified):
    Phi = T G T^T, entries below the keep-th largest |Phi| dropped.  transform:
    "block_dct8", "haar1", "haar1_lowpass" (high frequencies set to zero), "dct"
    (the full DCT-II) or "identity".  The threshold is the keep-th largest |Phi|
    (``keep``) or a given value (``eps``): exactly one of them.  Returns Y, or
    (Y, info dict with 'eps' and 'nnz' added)."""
    import torch
    m, n, ldx = _mat(X, "X")
    if out is None:
        out = torch.empty((m, n), device=X.device, dtype=torch.float32)
    _, _, ldy = _mat(out, "out")
    if tuple(out.shape) != (m, n):
        raise ValueError("out has the wrong shape")
    if (keep is None) == (eps is None):
        raise ValueError("give exactly one of keep and eps")
    if eps is None:
        sp = CpaSparsify(_TRANSFORMS[transform], THRESHOLD_KEEP, int(keep), 0.0)
    else:
        sp = CpaSparsify(_TRANSFORMS[transform], THRESHOLD_ABSOLUTE, 0, float(eps))
    ci = CpaInfo()
    eps = ctypes.c_double()
    nnz = ctypes.c_int64()
    co = opts.to_c()
    _check(lib().cpa_shrink_dense_sparsified(ctypes.c_void_p(context(X.device.index or 0)), _stream(X), m, n,
                                             ctypes.c_void_p(X.data_ptr()), ldx, ctypes.c_void_p(out.data_ptr()), ldy,
                                             ctypes.byref(shrink), ctypes.byref(co), ctypes.byref(sp),
                                             ctypes.byref(ci) if info else None, ctypes.byref(eps) if info else None,
                                             ctypes.byref(nnz) if info else None))
    if not info:
        return out
    d = ci.as_dict()
    d["eps"] = eps.value
    d["nnz"] = nnz.value
    return out, d


def _vec(t, name, dtype, count, device, nullable=True):
    """Checks a 1-D contiguous CUDA tensor of `dtype` with at least `count` entries."""
    import torch
    if t is None:
        if nullable:
            return
        raise TypeError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or t.device != device or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor on {device}")
    if t.numel() < count:
        raise ValueError(f"{name} holds {t.numel()} entries, {count} needed")


def _batch_args(X, m, n, off, out, shrink_per_matrix=None, Lambda=None, lambda_out=None, status=None,
                layout=True):
    """Type, device and length checks of a packed batch's tensors; with `layout`,
    also every matrix's extent against X and out (one host read of m, n, off)."""
    import torch
    if not isinstance(X, torch.Tensor) or not X.is_cuda or X.dtype != torch.float32 or not X.is_contiguous():
        raise TypeError("X must be a contiguous float32 CUDA tensor")
    dev = X.device
    if not isinstance(m, torch.Tensor) or m.dim() != 1:
        raise TypeError("m must be a 1-D int32 CUDA tensor")
    batch = int(m.numel())
    _vec(m, "m", torch.int32, batch, dev, False)
    _vec(n, "n", torch.int32, batch, dev, False)
    _vec(off, "off", torch.int64, batch, dev, False)
    _vec(out, "out", torch.float32, X.numel(), dev, False)
    _vec(shrink_per_matrix, "shrink_per_matrix", torch.uint8, batch * ctypes.sizeof(CpaShrinkage), dev)
    _vec(Lambda, "Lambda", torch.float64, batch, dev)
    _vec(lambda_out, "lambda_out", torch.float64, batch, dev)
    _vec(status, "status", torch.int32, batch, dev)
    if layout and batch > 0:
        mh = m.cpu().numpy().astype(np.int64)
        nh = n.cpu().numpy().astype(np.int64)
        oh = off.cpu().numpy()
        if (mh < 0).any() or (nh < 0).any() or (oh < 0).any():
            raise ValueError("negative size or offset in the batch")
        if (oh + mh * nh > X.numel()).any():
            raise ValueError("a matrix of the batch extends past the end of X")
    return batch


def shrink_batched(X, m, n, off, shrink, opts: Opts, shrink_per_matrix=None, Lambda=None, out=None,
                   lambda_out=None, status=None, check_layout: bool = True):
    """Shrinks every matrix of a packed batch (see cpa_shrink_batched).

    X: 1-D float32 CUDA tensor; m, n: int32 CUDA tensors; off: int64 CUDA tensor.
    shrink_per_matrix: optional uint8 CUDA tensor holding `batch` packed
    cpa_shrinkage records (see shrinkage_records).  check_layout reads m, n and off
    to the host to check every matrix lies inside X.  Returns Y."""
    import torch
    if out is None and isinstance(X, torch.Tensor):
        out = torch.empty_like(X)
    batch = _batch_args(X, m, n, off, out, shrink_per_matrix, Lambda, lambda_out, status, check_layout)
    co = opts.to_c()
    _check(lib().cpa_shrink_batched(ctypes.c_void_p(context(X.device.index or 0)), _stream(X), batch, _ptr(m),
                                    _ptr(n), _ptr(off), _ptr(X), _ptr(out), _ptr(shrink_per_matrix),
                                    ctypes.byref(shrink), ctypes.byref(co), _ptr(Lambda), _ptr(lambda_out),
                                    _ptr(status)))
    return out


class BatchedPlan:
    """A packed batch bound to one captured, tuned launch (see cpa_batched_plan_create).

    Takes the arguments of shrink_batched and keeps references to every tensor;
    `run()` replays the graph on the current stream and returns `out`.  The
    shapes (m, n, off) must not change; X, Lambda and the per-matrix records may."""

    def __init__(self, X, m, n, off, shrink, opts: Opts, shrink_per_matrix=None, Lambda=None, out=None,
                 lambda_out=None, status=None, tune: bool = True):
        import torch
        if out is None and isinstance(X, torch.Tensor):
            out = torch.empty_like(X)
        _batch_args(X, m, n, off, out, shrink_per_matrix, Lambda, lambda_out, status)
        self._h = None
        self._keep = (X, m, n, off, shrink_per_matrix, Lambda, out, lambda_out, status)
        self._shrink = shrink
        self._co = opts.to_c()
        self.out = out
        self.device = X.device
        h = ctypes.c_void_p()
        _check(lib().cpa_batched_plan_create(ctypes.c_void_p(context(X.device.index or 0)), _stream(X),
                                             int(m.numel()), _ptr(m), _ptr(n), _ptr(off), _ptr(X), _ptr(out),
                                             _ptr(shrink_per_matrix), ctypes.byref(self._shrink),
                                             ctypes.byref(self._co), _ptr(Lambda), _ptr(lambda_out), _ptr(status),
                                             1 if tune else 0, ctypes.byref(h)))
        self._h = h.value
        _plans.add(self)

    def run(self):
        if self._h is None:
            raise RuntimeError("plan is closed")
        _check(lib().cpa_batched_plan_execute(ctypes.c_void_p(self._h), _stream(self.out)))
        return self.out

    @property
    def tuning(self) -> dict:
        t = CpaBatchedTuning()
        _check(lib().cpa_batched_plan_tuning(ctypes.c_void_p(self._h), ctypes.byref(t)))
        return {"grid": t.grid, "pair": t.pair, "order": ("index", "largest_first")[t.order],
                "candidates": t.candidates, "best_us": t.best_us, "default_us": t.default_us}

    def close(self):
        if self._h is not None:
            _check(lib().cpa_batched_plan_destroy(ctypes.c_void_p(self._h)))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PRED_PARAMS = 4546
PRED_MODEL_FLOATS = 4554


def batched_features(X, m, n, off, out=None, status=None):
    """Predictor features (batch x 3 float32) of every matrix of a packed batch."""
    import torch
    batch = int(m.numel())
    if out is None:
        out = torch.empty((batch, 3), device=X.device, dtype=torch.float32)
    _batch_args(X, m, n, off, X, status=status)
    _vec(out, "out", torch.float32, 3 * batch, X.device, False)
    _check(lib().cpa_batched_features(ctypes.c_void_p(context(X.device.index or 0)), _stream(X), batch, _ptr(m),
                                      _ptr(n), _ptr(off), _ptr(X), _ptr(out), _ptr(status)))
    return out


def shrink_batched_predicted(X, m, n, off, shrink, opts: Opts, model, K_min: int = 2, shrink_per_matrix=None,
                             out=None, lambda_out=None, K_out=None, status=None):
    """Batched shrinkage with Lambda and K_j from the predictor `model` (float32 CUDA
    tensor of PRED_MODEL_FLOATS entries); opts.K is the largest order."""
    import torch
    if out is None and isinstance(X, torch.Tensor):
        out = torch.empty_like(X)
    batch = _batch_args(X, m, n, off, out, shrink_per_matrix, None, lambda_out, status)
    _vec(K_out, "K_out", torch.int32, batch, X.device)
    if not isinstance(model, torch.Tensor) or model.device != X.device or model.dtype != torch.float32 \
            or model.numel() != PRED_MODEL_FLOATS or not model.is_contiguous():
        raise ValueError("model must be a contiguous float32 tensor of %d entries on X's device" % PRED_MODEL_FLOATS)
    co = opts.to_c()
    _check(lib().cpa_shrink_batched_predicted(ctypes.c_void_p(context(X.device.index or 0)), _stream(X), batch,
                                              _ptr(m), _ptr(n), _ptr(off), _ptr(X), _ptr(out),
                                              _ptr(shrink_per_matrix), ctypes.byref(shrink), ctypes.byref(co),
                                              _ptr(model), int(K_min), _ptr(lambda_out), _ptr(K_out), _ptr(status)))
    return out


def _quantiles(q):
    return (ctypes.c_float * 2)(float(q[0]), float(q[1]))


def predictor_forward(feat, model, out=None):
    """Network outputs (n x 2) for feature rows feat (n x 3), both float32 CUDA tensors."""
    import torch
    n = int(feat.shape[0])
    if out is None:
        out = torch.empty((n, 2), device=feat.device, dtype=torch.float32)
    _check(lib().cpa_predictor_forward(ctypes.c_void_p(context(feat.device.index or 0)), _stream(feat), n,
                                       _ptr(feat.contiguous()), _ptr(model), _ptr(out)))
    return out


def predictor_grad(feat, targ, model, quantiles=(0.99, 0.9)):
    """(gradient (PRED_PARAMS float32), loss (float64 tensor of 1)) of the pinball loss."""
    import torch
    n = int(feat.shape[0])
    grad = torch.empty(PRED_PARAMS, device=feat.device, dtype=torch.float32)
    loss = torch.empty(1, device=feat.device, dtype=torch.float64)
    _check(lib().cpa_predictor_grad(ctypes.c_void_p(context(feat.device.index or 0)), _stream(feat), n,
                                    _ptr(feat), _ptr(targ), _quantiles(quantiles), _ptr(model), _ptr(grad),
                                    _ptr(loss)))
    return grad, loss


def predictor_train(feat, targ, model, adam_state, step: int, quantiles=(0.99, 0.9), batch_size: int = 1024,
                    epochs: int = 1, lr: float = 1e-3, epoch_loss=None):
    """Runs `epochs` passes of minibatch Adam on `model` in place; returns the new step count."""
    n = int(feat.shape[0])
    st = ctypes.c_int64(int(step))
    _check(lib().cpa_predictor_train(ctypes.c_void_p(context(feat.device.index or 0)), _stream(feat), n,
                                     _ptr(feat), _ptr(targ), _quantiles(quantiles), int(batch_size), int(epochs),
                                     float(lr), _ptr(model), _ptr(adam_state), ctypes.byref(st),
                                     _ptr(epoch_loss)))
    return int(st.value)


def shrink_csr(m, n, rowptr, colidx, vals, shrink, opts: Opts, out=None, info: bool = False):
    """Dense hat G(S) of a CSR matrix (int32 rowptr/colidx, float32 vals, CUDA tensors)."""
    import torch
    if out is None:
        out = torch.empty((m, n), device=vals.device, dtype=torch.float32)
    _, _, ldy = _mat(out, "out")
    ci = CpaInfo()
    co = opts.to_c()
    _check(lib().cpa_shrink_csr(ctypes.c_void_p(context(vals.device.index or 0)), _stream(vals), int(m), int(n),
                                int(vals.numel()), _ptr(rowptr), _ptr(colidx), _ptr(vals), _ptr(out), ldy,
                                ctypes.byref(shrink), ctypes.byref(co), ctypes.byref(ci) if info else None))
    return (out, ci.as_dict()) if info else out


def svt_complete(m, n, rowptr, colidx, mvals, tau: float, delta: float, iters: int, opts: Opts, out=None,
                 resid=None, y_start=None, y_end=None, lambdas=None):
    """SVT matrix completion on the observed CSR entries; returns (X, k0).

    y_start / y_end: float32 CUDA tensors of nnz values (the iterate on the
    observed set, CSR order) to continue from / to receive the final iterate;
    lambdas: float64 CUDA tensor of `iters` entries for each iteration's bound."""
    import torch
    if out is None:
        out = torch.empty((m, n), device=mvals.device, dtype=torch.float32)
    _, _, ldx = _mat(out, "out")
    nnz = int(mvals.numel())
    _vec(y_start, "y_start", torch.float32, nnz, mvals.device)
    _vec(y_end, "y_end", torch.float32, nnz, mvals.device)
    _vec(lambdas, "lambdas", torch.float64, int(iters), mvals.device)
    _vec(resid, "resid", torch.float64, int(iters), mvals.device)
    k0 = ctypes.c_double()
    co = opts.to_c()
    _check(lib().cpa_svt_complete(ctypes.c_void_p(context(mvals.device.index or 0)), _stream(mvals), int(m), int(n),
                                  nnz, _ptr(rowptr), _ptr(colidx), _ptr(mvals), float(tau),
                                  float(delta), int(iters), _ptr(out), ldx, ctypes.byref(co), _ptr(resid),
                                  ctypes.byref(k0), _ptr(y_start), _ptr(y_end), _ptr(lambdas)))
    return out, k0.value


def shrinkage_records(records) -> bytes:
    """Packs a list of CpaShrinkage into the byte layout of a cpa_shrinkage array."""
    return b"".join(bytes(r) for r in records)


def workspace_bytes(m: int, n: int, opts: Opts, device: int = 0) -> int:
    """Device bytes the dense shrink of an m x n input needs (see cpa_workspace_bytes)."""
    out = ctypes.c_size_t()
    co = opts.to_c()
    _check(lib().cpa_workspace_bytes(ctypes.c_void_p(context(device)), int(m), int(n), ctypes.byref(co),
                                     ctypes.byref(out)))
    return int(out.value)


def peak_mfma(kind: str = "fp32", iters: int = 4000, device: int = 0, clock: bool = False):
    """Achievable dense MFMA rate of the device in TFLOP/s (see cpa_peak_mfma);
    with clock=True, (rate, shader clock in GHz during the MFMA loop)."""
    import torch
    out = ctypes.c_double()
    ghz = ctypes.c_double()
    _check(lib().cpa_peak_mfma(ctypes.c_void_p(context(device)),
                               ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream),
                               {"fp32": 0, "bf16": 1}[kind], int(iters), ctypes.byref(out),
                               ctypes.byref(ghz) if clock else None))
    return (out.value, ghz.value) if clock else out.value


def timing_enable(enable: bool = True, device: int = 0):
    """Start (or stop) per-launch event timing of the GEMM kernels; resets the record."""
    _check(lib().cpa_timing_enable(ctypes.c_void_p(context(device)), int(bool(enable))))


def timing_read(which: str = "recurrence", device: int = 0):
    """(total kernel milliseconds, launches) recorded since timing_enable."""
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(lib().cpa_timing_read(ctypes.c_void_p(context(device)), {"recurrence": 0, "gram": 1, "pieces": 2}[which],
                                 ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def rpca_admm(I, inv_rho: float, eta_over_rho: float, max_iters: int, tol: float, opts: Opts):
    """RPCA by ADMM in one call (cpa_rpca_admm): returns (L, S, E_t list, iterations)."""
    import torch
    m, n, ld = _mat(I, "I")
    if ld != n:
        raise ValueError("I must be contiguous")
    L = torch.empty((m, n), device=I.device, dtype=torch.float32)
    S = torch.empty_like(L)
    Et = (ctypes.c_double * max(int(max_iters), 1))()
    done = ctypes.c_int()
    co = opts.to_c()
    _check(lib().cpa_rpca_admm(ctypes.c_void_p(context(I.device.index or 0)), _stream(I), m, n,
                               ctypes.c_void_p(I.data_ptr()), ctypes.c_void_p(L.data_ptr()),
                               ctypes.c_void_p(S.data_ptr()), float(inv_rho), float(eta_over_rho), int(max_iters),
                               float(tol), ctypes.byref(co), Et, ctypes.byref(done)))
    return L, S, list(Et[:done.value]), done.value


class Inpaint:
    """Texture inpainting by ADMM (Appendix A of the paper) with CPA shrinkage,
    state on the device (see cpa_inpaint_iterate).  ``omega``: 1 on the observed
    pixels, 0 on the region to recover; ``border``: 1 on the surrounding pixels
    whose mean the region is held to, or None for no mean term.  ``state`` holds
    the blocks [l, z1..z5, u1..u5]; ``L`` views the first."""

    NAMES = ("l", "z1", "z2", "z3", "z4", "z5", "u1", "u2", "u3", "u4", "u5")

    def __init__(self, I, omega, inv_rho: float, eta_over_rho: float, opts: Opts, border=None):
        import torch
        m, n, ld = _mat(I, "I")
        if ld != n:
            raise ValueError("I must be contiguous")
        self.I, self.m, self.n = I, m, n
        self.omega = omega.to(device=I.device, dtype=torch.float32).contiguous()
        self.border = None if border is None else border.to(device=I.device, dtype=torch.float32).contiguous()
        for t in (self.omega, self.border):
            if t is not None and tuple(t.shape) != (m, n):
                raise ValueError("omega and border must have the shape of I")
        self.inv_rho, self.eta_over_rho, self.opts = float(inv_rho), float(eta_over_rho), opts
        count = lib().cpa_inpaint_state_floats(m, n)
        self.state = torch.empty(count, device=I.device, dtype=torch.float32)
        self.dev_index = I.device.index or 0
        _check(lib().cpa_inpaint_init(ctypes.c_void_p(context(self.dev_index)), _stream(I), m, n,
                                      ctypes.c_void_p(self.omega.data_ptr()), ctypes.c_void_p(self.state.data_ptr())))

    def block(self, i: int):
        mn = self.m * self.n
        return self.state[i * mn:(i + 1) * mn].view(self.m, self.n)

    @property
    def L(self):
        return self.block(0)

    def iterate(self, iters: int, Et=None):
        """Runs ``iters`` iterations; ``Et`` (float64 CUDA tensor, >= iters) receives E_t."""
        co = self.opts.to_c()
        ptr = ctypes.c_void_p(Et.data_ptr()) if Et is not None else None
        bptr = ctypes.c_void_p(self.border.data_ptr()) if self.border is not None else None
        _check(lib().cpa_inpaint_iterate(ctypes.c_void_p(context(self.dev_index)), _stream(self.I), self.m, self.n,
                                         ctypes.c_void_p(self.I.data_ptr()), ctypes.c_void_p(self.omega.data_ptr()),
                                         bptr, ctypes.c_void_p(self.state.data_ptr()), int(iters), self.inv_rho,
                                         self.eta_over_rho, ctypes.byref(co), ptr))


    def iterate_scheduled(self, iters: int, Et, transform: str = "dct", E_prev: float = float("inf"),
                          E_l: float = SCHEDULE_E_L, E_m: float = SCHEDULE_E_M):
        """Runs ``iters`` iterations with z1 by the sparsified shrink and the keep
        count of eq. (recommendation_epsilon) from the previous E_t (E_prev before
        the first); ``Et`` (float64 CUDA tensor, >= iters) is required.  Returns the
        keep counts (cpa_inpaint_iterate_scheduled)."""
        if Et is None or Et.numel() < iters:
            raise ValueError("Et must hold iters float64 values")
        co = self.opts.to_c()
        keeps = (ctypes.c_int64 * max(int(iters), 1))()
        bptr = ctypes.c_void_p(self.border.data_ptr()) if self.border is not None else None
        _check(lib().cpa_inpaint_iterate_scheduled(
            ctypes.c_void_p(context(self.dev_index)), _stream(self.I), self.m, self.n, ctypes.c_void_p(self.I.data_ptr()),
            ctypes.c_void_p(self.omega.data_ptr()), bptr, ctypes.c_void_p(self.state.data_ptr()), int(iters),
            self.inv_rho, self.eta_over_rho, ctypes.byref(co), _TRANSFORMS[transform], float(E_prev), float(E_l),
            float(E_m), ctypes.c_void_p(Et.data_ptr()), keeps))
        return [int(k) for k in keeps[:int(iters)]]


class RpcaAdmm:
    """RPCA by ADMM (Appendix B of the paper) with CPA shrinkage, state on the device.

    ``state`` holds the blocks [l, s, z1, z2, u1, u2, u3]; ``L`` and ``S`` view
    the first two."""

    def __init__(self, I, inv_rho: float, eta_over_rho: float, opts: Opts):
        import torch
        m, n, ld = _mat(I, "I")
        if ld != n:
            raise ValueError("I must be contiguous")
        self.I, self.m, self.n = I, m, n
        self.inv_rho, self.eta_over_rho, self.opts = float(inv_rho), float(eta_over_rho), opts
        count = lib().cpa_rpca_state_floats(m, n)
        self.state = torch.empty(count, device=I.device, dtype=torch.float32)
        self.dev_index = I.device.index or 0
        self.t = 0
        _check(lib().cpa_rpca_init(ctypes.c_void_p(context(self.dev_index)), _stream(I), m, n,
                                   ctypes.c_void_p(self.state.data_ptr())))

    def block(self, i: int):
        mn = self.m * self.n
        return self.state[i * mn:(i + 1) * mn].view(self.m, self.n)

    @property
    def L(self):
        return self.block(0)

    @property
    def S(self):
        return self.block(1)

    def iterate(self, iters: int, Et=None):
        """Runs ``iters`` iterations; ``Et`` (float64 CUDA tensor, >= iters) receives E_t."""
        co = self.opts.to_c()
        ptr = ctypes.c_void_p(Et.data_ptr()) if Et is not None else None
        _check(lib().cpa_rpca_iterate(ctypes.c_void_p(context(self.dev_index)), _stream(self.I), self.m, self.n,
                                      ctypes.c_void_p(self.I.data_ptr()), ctypes.c_void_p(self.state.data_ptr()),
                                      int(iters), self.inv_rho, self.eta_over_rho, ctypes.byref(co), ptr))
        self.t += iters
