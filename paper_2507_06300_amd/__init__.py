"""MI355X batched flexible-PSD / Whittle log-likelihood (arXiv 2507.06300 hot path).

A thin ctypes binding over the C ABI of ``liblps.so`` (declared in
``include/lps.h``).  PyTorch provides device memory and streams only; every
step of the computation runs in the library's HIP kernels.  The names follow
the ABI: ``psd_build``, ``loglike_batch``, ``loglike_grad_batch``,
``loglike_plain_fp64``.  If the library is missing the import fails loudly:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblps.so")

FP64 = 0
MIXED = 1
_PREC = {"fp64": FP64, "mixed": MIXED, FP64: FP64, MIXED: MIXED}

ST_COUNT, ST_ORDER, ST_COVER, ST_NONFINITE, ST_AMPLITUDE, ST_PSD = 1, 2, 4, 8, 16, 32

_STATUS_NAMES = {0: "LPS_OK", 1: "LPS_E_NULL", 2: "LPS_E_SHAPE", 3: "LPS_E_CAPACITY", 4: "LPS_E_ROUTING",
                 5: "LPS_E_PRECISION", 6: "LPS_E_DEVICE", 7: "LPS_E_NOMEM", 8: "LPS_E_STATE",
                 9: "LPS_E_DATA"}


class LpsError(RuntimeError):
    def __init__(self, code, where, detail=None):
        self.code = code
        msg = f"{where}: {_STATUS_NAMES.get(code, code)} ({lib().lps_strerror(code).decode()})"
        super().__init__(msg + (f": {detail}" if detail else ""))


class _Desc(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("f", ctypes.c_void_p), ("nk", ctypes.c_void_p),
                ("D", ctypes.c_void_p), ("R", ctypes.c_void_p), ("Rfg", ctypes.c_void_p),
                ("f_knee", ctypes.c_double), ("arm_length", ctypes.c_double), ("n_spl", ctypes.c_int32),
                ("route", ctypes.c_int8 * 12), ("k_max", ctypes.c_int32), ("max_states", ctypes.c_int32),
                ("max_grad_states", ctypes.c_int32)]


class _CovDesc(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("f", ctypes.c_void_p), ("nk", ctypes.c_void_p),
                ("P", ctypes.c_void_p), ("R", ctypes.c_void_p), ("Rfg", ctypes.c_void_p),
                ("f_knee", ctypes.c_double), ("arm_length", ctypes.c_double), ("n_spl", ctypes.c_int32),
                ("route", ctypes.c_int8 * 12), ("corr", ctypes.c_int8 * 3), ("k_max", ctypes.c_int32),
                ("max_states", ctypes.c_int32)]


class _SamplerDesc(ctypes.Structure):
    _fields_ = [("n_walkers", ctypes.c_int32), ("n_temps", ctypes.c_int32), ("betas", ctypes.c_void_p),
                ("temp_scales", ctypes.c_void_p), ("seed", ctypes.c_uint64), ("k_in_max", ctypes.c_int32),
                ("step", ctypes.c_double), ("precision", ctypes.c_int), ("fixed_params", ctypes.c_uint32),
                ("rj_moves", ctypes.c_int32), ("stretch_moves", ctypes.c_int32)]


class _States(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_int32), ("params", ctypes.c_void_p), ("knot_off", ctypes.c_void_p),
                ("knot_x", ctypes.c_void_p), ("knot_y", ctypes.c_void_p), ("knot_cnt", ctypes.c_void_p),
                ("n_knots", ctypes.c_int64)]


SYMBOLS = ["lps_create", "lps_destroy", "lps_psd_build", "lps_loglike_batch", "lps_loglike_grad_batch",
           "lps_loglike_plain_fp64", "lps_set_timing", "lps_kernel_time_ms", "lps_get_error", "lps_strerror",
           "lps_chunk_bins", "lps_last_device_error", "lps_valu_probe", "lps_set_launch", "lps_get_launch", "lps_autotune",
           "lps_sampler_create", "lps_sampler_destroy", "lps_sampler_set_state", "lps_sampler_sweep",
           "lps_sampler_get_state", "lps_sampler_counters", "lps_philox4x32_10",
           "lps_stepping_stone", "lps_dic",
           "lps_data_periodogram", "lps_data_average", "lps_data_response",
           "lps_cov_create", "lps_cov_destroy", "lps_cov_loglike_batch", "lps_cov_loglike_grad_batch", "lps_cov_build",
           "lps_math64_check", "lps_loglike_plain_fp64_noalloc",
           "lps_data_create", "lps_data_destroy", "lps_data_periodogram_planned", "lps_paper_ladder",
           "lps_column_median"]

_lib = None


def lib():
    """Load liblps.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2507_06300_amd.build_lib.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int
    L.lps_create.argtypes = [ctypes.POINTER(_Desc), ctypes.c_int, ctypes.POINTER(vp)]
    L.lps_destroy.argtypes = [vp]
    L.lps_psd_build.argtypes = [vp, ctypes.POINTER(_States), i32, i32, vp, vp, vp, vp, vp]
    L.lps_loglike_batch.argtypes = [vp, ctypes.POINTER(_States), ctypes.c_int, vp, vp, vp]
    L.lps_loglike_grad_batch.argtypes = [vp, ctypes.POINTER(_States), ctypes.c_int, vp, vp, vp, vp, vp, vp]
    L.lps_loglike_plain_fp64.argtypes = [vp, ctypes.POINTER(_States), vp, vp, vp]
    L.lps_set_timing.argtypes = [vp, ctypes.c_int]
    L.lps_kernel_time_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
    L.lps_get_error.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_uint32)]
    L.lps_strerror.argtypes = [ctypes.c_int]
    L.lps_strerror.restype = ctypes.c_char_p
    L.lps_last_device_error.argtypes = [ctypes.POINTER(ctypes.c_char_p)]
    L.lps_last_device_error.restype = ctypes.c_int32
    L.lps_chunk_bins.argtypes = [ctypes.c_int]
    L.lps_chunk_bins.restype = ctypes.c_int32
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    L.lps_valu_probe.argtypes = [ctypes.c_int, dp, dp, dp]
    L.lps_valu_probe.restype = st
    L.lps_set_launch.argtypes = [vp, ctypes.c_int, i32, i32]
    L.lps_set_launch.restype = st
    L.lps_get_launch.argtypes = [vp, ctypes.c_int, i32, ip, ip]
    L.lps_get_launch.restype = st
    L.lps_autotune.argtypes = [vp, ctypes.POINTER(_States), ctypes.c_int, i32, dp, vp]
    L.lps_autotune.restype = st
    L.lps_sampler_create.argtypes = [vp, ctypes.POINTER(_SamplerDesc), ctypes.POINTER(vp)]
    L.lps_sampler_destroy.argtypes = [vp]
    L.lps_sampler_set_state.argtypes = [vp, ctypes.POINTER(_States), ctypes.c_uint64, vp]
    L.lps_sampler_sweep.argtypes = [vp, i32, vp]
    L.lps_sampler_get_state.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_uint64), vp]
    L.lps_sampler_counters.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32), vp]
    L.lps_philox4x32_10.argtypes = [ctypes.c_uint64, ctypes.c_uint64, i32, vp, vp]
    L.lps_stepping_stone.argtypes = [vp, i32, vp, i32, i32, vp, vp]
    L.lps_dic.argtypes = [vp, i32, i32, i32, i32, vp, vp, vp]
    L.lps_data_periodogram.argtypes = [vp, i32, i32, ctypes.c_double, vp, i32, vp, vp]
    L.lps_data_average.argtypes = [vp, i32, i32, vp, i32, i32, i32, vp, vp, vp, vp]
    L.lps_data_response.argtypes = [vp, vp, i32, i32, vp, i32, vp, vp]
    L.lps_cov_create.argtypes = [ctypes.POINTER(_CovDesc), ctypes.c_int, ctypes.POINTER(vp)]
    L.lps_cov_destroy.argtypes = [vp]
    L.lps_cov_loglike_batch.argtypes = [vp, ctypes.POINTER(_States), vp, vp, vp]
    L.lps_cov_loglike_grad_batch.argtypes = [vp, ctypes.POINTER(_States), vp, vp, vp, vp, vp, vp]
    L.lps_cov_build.argtypes = [vp, ctypes.POINTER(_States), i32, i32, vp, vp, vp]
    L.lps_math64_check.argtypes = [vp, i32, i32, vp, vp]
    L.lps_loglike_plain_fp64_noalloc.argtypes = [ctypes.POINTER(_Desc), ctypes.POINTER(_States), vp, vp, vp]
    L.lps_data_create.argtypes = [i32, i32, ctypes.c_int, ctypes.POINTER(vp)]
    L.lps_data_destroy.argtypes = [vp]
    L.lps_data_periodogram_planned.argtypes = [vp, vp, ctypes.c_double, vp, i32, vp, vp]
    L.lps_paper_ladder.argtypes = [vp]
    L.lps_column_median.argtypes = [vp, i32, i32, i32, vp, vp]
    for name in ["lps_sampler_create", "lps_sampler_destroy", "lps_sampler_set_state", "lps_sampler_sweep",
                 "lps_sampler_get_state", "lps_sampler_counters", "lps_philox4x32_10", "lps_stepping_stone",
                 "lps_dic", "lps_data_periodogram", "lps_data_average", "lps_data_response",
                 "lps_cov_create", "lps_cov_destroy", "lps_cov_loglike_batch", "lps_cov_loglike_grad_batch",
                 "lps_cov_build", "lps_math64_check", "lps_loglike_plain_fp64_noalloc", "lps_data_create",
                 "lps_data_destroy", "lps_data_periodogram_planned", "lps_paper_ladder", "lps_column_median"]:
        getattr(L, name).restype = st
    for name in ["lps_create", "lps_destroy", "lps_psd_build", "lps_loglike_batch", "lps_loglike_grad_batch",
                 "lps_loglike_plain_fp64", "lps_set_timing", "lps_kernel_time_ms", "lps_get_error"]:
        getattr(L, name).restype = st
    _lib = L
    return L


# Handles whose release was postponed because the calling thread was capturing
# a graph: the destroy calls synchronise and free device memory, which would
# invalidate the capture (a garbage-collected Context can be finalised at any
# point, including inside a capture).
_DEFERRED = []


def _capturing():
    try:
        return torch.cuda.is_available() and torch.cuda.is_current_stream_capturing()
    except Exception:
        return False


def _release(destroy, h):
    _DEFERRED.append((destroy, h))
    _drain()


def _drain():
    if _capturing():
        return
    while _DEFERRED:
        destroy, h = _DEFERRED.pop(0)
        getattr(lib(), destroy)(h)


def _check(code, where):
    if code != 0:
        detail = None
        if code == 6:   # LPS_E_DEVICE: name the HIP error behind it
            name = ctypes.c_char_p()
            err = lib().lps_last_device_error(ctypes.byref(name))
            detail = f"HIP error {err} ({name.value.decode() if name.value else '?'})"
        raise LpsError(code, where, detail)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(a, dtype, device):
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=dtype)
    else:
        t = torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)
    return t.contiguous()


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def loglike_plain_fp64_noalloc(f, nk, D, R, route, n_spl, st: "States", Rfg=None, k_max=64, f_knee=1.0e-3,
                               arm_length=2.5e9, logL=None, status=None, stream=None):
    """lps_loglike_plain_fp64_noalloc: the plain FP64 path without a context.

    f, nk, D, R (and Rfg) must already be contiguous float64 device tensors;
    the call itself allocates nothing on the device (outputs are allocated
    here only when not given)."""
    for t in (f, nk, D, R) + (() if Rfg is None else (Rfg,)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise TypeError("dataset arrays must be contiguous float64 device tensors")
    n = st.n
    logL = logL if logL is not None else torch.empty(n, dtype=torch.float64, device=f.device)
    status = status if status is not None else torch.empty(n, dtype=torch.int32, device=f.device)
    d = _Desc()
    d.n_bins = int(f.numel())
    d.f, d.nk, d.D, d.R = f.data_ptr(), nk.data_ptr(), D.data_ptr(), R.data_ptr()
    d.Rfg = None if Rfg is None else Rfg.data_ptr()
    d.f_knee = float(f_knee)
    d.arm_length = float(arm_length)
    d.n_spl = int(n_spl)
    flat = [int(v) for row in route for v in row]
    for i in range(12):
        d.route[i] = flat[i]
    d.k_max = int(k_max)
    c = st._c()
    _check(lib().lps_loglike_plain_fp64_noalloc(ctypes.byref(d), ctypes.byref(c), _ptr(logL), _ptr(status),
                                                _stream(stream)), "lps_loglike_plain_fp64_noalloc")
    return logL, status


@dataclass
class States:
    """A state batch resident on the device (params [P][n], CSR knots).

    knot_cnt = None: packed CSR (counts are offset differences); otherwise a
    padded layout where spline i owns knot_cnt[i] knots from knot_off[i]."""
    params: torch.Tensor
    knot_off: torch.Tensor
    knot_x: torch.Tensor
    knot_y: torch.Tensor
    knot_cnt: Optional[torch.Tensor] = None

    @property
    def n(self) -> int:
        return int(self.params.shape[1])

    def _c(self):
        return _States(self.n, self.params.data_ptr(), self.knot_off.data_ptr(), self.knot_x.data_ptr(),
                       self.knot_y.data_ptr(), None if self.knot_cnt is None else self.knot_cnt.data_ptr(),
                       int(min(self.knot_x.numel(), self.knot_y.numel())))


class Context:
    """One analysed dataset on one GPU (wraps lps_create / lps_destroy)."""

    def __init__(self, f, nk, D, R, route, n_spl, Rfg=None, k_max=64, max_states=1, f_knee=1.0e-3,
                 arm_length=2.5e9, device=None, max_grad_states=None):
        _drain()
        self.device = torch.device(device if device is not None else "cuda")
        dev = self.device
        self.f = _dev(f, torch.float64, dev)
        self.nk = _dev(nk, torch.float64, dev)
        self.D = _dev(D, torch.float64, dev)
        self.R = _dev(R, torch.float64, dev)
        self.Rfg = None if Rfg is None else _dev(Rfg, torch.float64, dev)
        self.n_bins = int(self.f.numel())
        self.n_spl = int(n_spl)
        self.n_params = 5 if Rfg is not None else 4
        self.max_states = int(max_states)
        d = _Desc()
        d.n_bins = self.n_bins
        d.f, d.nk, d.D, d.R = (self.f.data_ptr(), self.nk.data_ptr(), self.D.data_ptr(), self.R.data_ptr())
        d.Rfg = None if self.Rfg is None else self.Rfg.data_ptr()
        d.f_knee = float(f_knee)
        d.arm_length = float(arm_length)
        d.n_spl = self.n_spl
        flat = [int(v) for row in route for v in row]
        for i in range(12):
            d.route[i] = flat[i]
        d.k_max = int(k_max)
        d.max_states = self.max_states
        self.max_grad_states = self.max_states if max_grad_states is None else int(max_grad_states)
        d.max_grad_states = self.max_grad_states
        h = ctypes.c_void_p()
        idx = dev.index if dev.index is not None else torch.cuda.current_device()
        _check(lib().lps_create(ctypes.byref(d), idx, ctypes.byref(h)), "lps_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _release("lps_destroy", self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def states(self, params, knot_off, knot_x, knot_y) -> States:
        dev = self.device
        kx, ky = _dev(knot_x, torch.float64, dev), _dev(knot_y, torch.float64, dev)
        if kx.numel() == 0:
            # a batch whose splines are all disabled holds no knots; the ABI still
            # wants non-NULL arrays (the offsets decide what is read: nothing)
            kx, ky = torch.zeros(1, dtype=torch.float64, device=dev), torch.zeros(1, dtype=torch.float64, device=dev)
        return States(_dev(params, torch.float64, dev), _dev(knot_off, torch.int32, dev), kx, ky)

    def psd_build(self, st: States, k0=0, k1=None, parts=False, stream=None):
        k1 = self.n_bins if k1 is None else int(k1)
        n = st.n
        S = torch.empty((n, 3, k1 - k0), dtype=torch.float64, device=self.device)
        Sn = torch.empty_like(S) if parts else None
        Sh = torch.empty_like(S) if parts else None
        status = torch.empty(n, dtype=torch.int32, device=self.device)
        c = st._c()
        _check(lib().lps_psd_build(self._h, ctypes.byref(c), int(k0), int(k1), _ptr(S), _ptr(Sn), _ptr(Sh),
                                   _ptr(status), _stream(stream)), "lps_psd_build")
        return (S, Sn, Sh, status) if parts else (S, status)

    def loglike_batch(self, st: States, precision="fp64", out=None, status=None, stream=None):
        n = st.n
        logL = out if out is not None else torch.empty(n, dtype=torch.float64, device=self.device)
        status = status if status is not None else torch.empty(n, dtype=torch.int32, device=self.device)
        c = st._c()
        _check(lib().lps_loglike_batch(self._h, ctypes.byref(c), _PREC.get(precision, precision), _ptr(logL), _ptr(status),
                                       _stream(stream)), "lps_loglike_batch")
        return logL, status

    def loglike_grad_batch(self, st: States, precision="fp64", stream=None):
        n = st.n
        logL = torch.empty(n, dtype=torch.float64, device=self.device)
        dparams = torch.empty((self.n_params, n), dtype=torch.float64, device=self.device)
        dkx = torch.empty_like(st.knot_x)
        dky = torch.empty_like(st.knot_y)
        status = torch.empty(n, dtype=torch.int32, device=self.device)
        c = st._c()
        _check(lib().lps_loglike_grad_batch(self._h, ctypes.byref(c), _PREC.get(precision, precision), _ptr(logL), _ptr(dparams),
                                            _ptr(dkx), _ptr(dky), _ptr(status), _stream(stream)),
               "lps_loglike_grad_batch")
        return logL, dparams, dkx, dky, status

    def loglike_plain_fp64(self, st: States, stream=None):
        n = st.n
        logL = torch.empty(n, dtype=torch.float64, device=self.device)
        status = torch.empty(n, dtype=torch.int32, device=self.device)
        c = st._c()
        _check(lib().lps_loglike_plain_fp64(self._h, ctypes.byref(c), _ptr(logL), _ptr(status), _stream(stream)),
               "lps_loglike_plain_fp64")
        return logL, status

    def set_launch(self, precision, bins_per_lane=0, states_per_tile=0):
        _check(lib().lps_set_launch(self._h, _PREC.get(precision, precision), int(bins_per_lane),
                                    int(states_per_tile)), "lps_set_launch")

    def get_launch(self, precision, n_states):
        b, t = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().lps_get_launch(self._h, _PREC.get(precision, precision), int(n_states), ctypes.byref(b),
                                    ctypes.byref(t)), "lps_get_launch")
        return b.value, t.value

    def autotune(self, st: States, precision="mixed", reps=3, stream=None):
        """Time the candidate launch shapes on this batch and keep the fastest."""
        ms = ctypes.c_double()
        c = st._c()
        _check(lib().lps_autotune(self._h, ctypes.byref(c), _PREC.get(precision, precision), int(reps),
                                  ctypes.byref(ms), _stream(stream)), "lps_autotune")
        return ms.value, self.get_launch(precision, st.n)

    def set_timing(self, on: bool):
        _check(lib().lps_set_timing(self._h, 1 if on else 0), "lps_set_timing")

    def kernel_time(self):
        ms = ctypes.c_double()
        n = ctypes.c_int32()
        _check(lib().lps_kernel_time_ms(self._h, ctypes.byref(ms), ctypes.byref(n)), "lps_kernel_time_ms")
        return ms.value, n.value

    def get_error(self, stream=None):
        v = ctypes.c_uint32()
        _check(lib().lps_get_error(self._h, _stream(stream), ctypes.byref(v)), "lps_get_error")
        return v.value


class CovContext:
    """Full-covariance (dense 3x3 A/E/T) likelihood for one dataset
    (wraps lps_cov_create / lps_cov_destroy).  P holds the six real
    cross-periodogram rows AA, EE, TT, AE, AT, ET; route is the diagonal
    routing [4][3] and corr the spline slots of the three correlation terms."""

    def __init__(self, f, nk, P, R, route, corr, n_spl, Rfg=None, k_max=64, max_states=1, f_knee=1.0e-3,
                 arm_length=2.5e9, device=None):
        _drain()
        self.device = torch.device(device if device is not None else "cuda")
        dev = self.device
        self.f = _dev(f, torch.float64, dev)
        self.nk = _dev(nk, torch.float64, dev)
        self.P = _dev(P, torch.float64, dev)
        self.R = _dev(R, torch.float64, dev)
        self.Rfg = None if Rfg is None else _dev(Rfg, torch.float64, dev)
        self.n_bins = int(self.f.numel())
        self.n_spl = int(n_spl)
        self.n_params = 4 if Rfg is None else 5
        self.max_states = int(max_states)
        d = _CovDesc()
        d.n_bins = self.n_bins
        d.f, d.nk, d.P, d.R = (self.f.data_ptr(), self.nk.data_ptr(), self.P.data_ptr(), self.R.data_ptr())
        d.Rfg = None if self.Rfg is None else self.Rfg.data_ptr()
        d.f_knee = float(f_knee)
        d.arm_length = float(arm_length)
        d.n_spl = self.n_spl
        flat = [int(v) for row in route for v in row]
        for i in range(12):
            d.route[i] = flat[i]
        for i in range(3):
            d.corr[i] = int(corr[i])
        d.k_max = int(k_max)
        d.max_states = self.max_states
        h = ctypes.c_void_p()
        idx = dev.index if dev.index is not None else torch.cuda.current_device()
        _check(lib().lps_cov_create(ctypes.byref(d), idx, ctypes.byref(h)), "lps_cov_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _release("lps_cov_destroy", self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def states(self, params, knot_off, knot_x, knot_y) -> States:
        dev = self.device
        kx, ky = _dev(knot_x, torch.float64, dev), _dev(knot_y, torch.float64, dev)
        if kx.numel() == 0:
            # a batch whose splines are all disabled holds no knots; the ABI still
            # wants non-NULL arrays (the offsets decide what is read: nothing)
            kx, ky = torch.zeros(1, dtype=torch.float64, device=dev), torch.zeros(1, dtype=torch.float64, device=dev)
        return States(_dev(params, torch.float64, dev), _dev(knot_off, torch.int32, dev), kx, ky)

    def loglike_batch(self, st: States, out=None, status=None, stream=None):
        n = st.n
        logL = out if out is not None else torch.empty(n, dtype=torch.float64, device=self.device)
        status = status if status is not None else torch.empty(n, dtype=torch.int32, device=self.device)
        c = st._c()
        _check(lib().lps_cov_loglike_batch(self._h, ctypes.byref(c), _ptr(logL), _ptr(status), _stream(stream)),
               "lps_cov_loglike_batch")
        return logL, status

    def loglike_grad_batch(self, st: States, stream=None):
        """logL, dlogL/dparams [n_params][n], dlogL/dknot_x, dlogL/dknot_y (the
        states' CSR layout) and status."""
        n = st.n
        logL = torch.empty(n, dtype=torch.float64, device=self.device)
        dparams = torch.empty((self.n_params, n), dtype=torch.float64, device=self.device)
        dkx = torch.empty_like(st.knot_x)
        dky = torch.empty_like(st.knot_y)
        status = torch.empty(n, dtype=torch.int32, device=self.device)
        c = st._c()
        _check(lib().lps_cov_loglike_grad_batch(self._h, ctypes.byref(c), _ptr(logL), _ptr(dparams), _ptr(dkx),
                                                _ptr(dky), _ptr(status), _stream(stream)),
               "lps_cov_loglike_grad_batch")
        return logL, dparams, dkx, dky, status

    def build(self, st: States, k0=0, k1=None, stream=None):
        """Model covariance rows C[s][6][k1 - k0] (AA, EE, TT, AE, AT, ET) and status."""
        k1 = self.n_bins if k1 is None else int(k1)
        n = st.n
        C = torch.empty((n, 6, k1 - int(k0)), dtype=torch.float64, device=self.device)
        status = torch.empty(n, dtype=torch.int32, device=self.device)
        c = st._c()
        _check(lib().lps_cov_build(self._h, ctypes.byref(c), int(k0), int(k1), _ptr(C), _ptr(status),
                                   _stream(stream)), "lps_cov_build")
        return C, status


MATH64 = {"exp2": 0, "log2": 1, "rcp": 2, "sqrt": 3, "log": 4, "exp2_table": 5, "rsq": 6}


def math64_check(fn: str, x, stream=None):
    """The library's FP64 elementary function `fn` (see MATH64) applied to x on the device."""
    xd = _dev(x, torch.float64, torch.device("cuda"))
    out = torch.empty_like(xd)
    _check(lib().lps_math64_check(_ptr(xd), int(xd.numel()), MATH64[fn], _ptr(out), _stream(stream)),
           "lps_math64_check")
    return out


def valu_probe(device=0):
    """(ns per wave64 FMA per SIMD, transcendental cost in FMA slots, lane-instr/s)."""
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().lps_valu_probe(int(device), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "lps_valu_probe")
    return a.value, b.value, c.value


def chunk_bins(precision="fp64") -> int:
    return int(lib().lps_chunk_bins(_PREC.get(precision, precision)))


def philox4x32_10(seed: int, first_counter: int, n: int, device="cuda"):
    """The sampler's generator on the device: uint32 [n][4] (as int64 tensor)."""
    out = torch.empty(4 * n, dtype=torch.int32, device=device)
    _check(lib().lps_philox4x32_10(ctypes.c_uint64(seed), ctypes.c_uint64(first_counter), int(n), _ptr(out),
                                   _stream(None)), "lps_philox4x32_10")
    return (out.to(torch.int64) & 0xFFFFFFFF).view(n, 4)


def data_periodogram(x: torch.Tensor, dt, window=None, xyz_to_aet=False, stream=None):
    """One-sided periodogram of time series x [n_ch, n_t] (device FP64): returns
    (f [n_t//2 + 1], P [n_ch, n_t//2 + 1]) on the device."""
    xs = _dev(x, torch.float64, x.device)
    n_ch, n_t = xs.shape
    w = None if window is None else _dev(window, torch.float64, xs.device)
    nf = n_t // 2 + 1
    P = torch.empty((n_ch, nf), dtype=torch.float64, device=xs.device)
    _check(lib().lps_data_periodogram(_ptr(xs), int(n_ch), int(n_t), float(dt), _ptr(w), 1 if xyz_to_aet else 0,
                                      _ptr(P), _stream(stream)), "lps_data_periodogram")
    f = torch.arange(nf, dtype=torch.float64, device=xs.device) / (n_t * float(dt))
    return f, P


class DataPlan:
    """A planned periodogram of n_ch series of n_t samples (wraps lps_data_create /
    lps_data_destroy): the transform plan and temporaries are made once, so that
    periodogram() is asynchronous, allocates nothing on the device itself and may
    be captured into a HIP graph."""

    def __init__(self, n_ch, n_t, device=None):
        _drain()
        self.device = torch.device(device if device is not None else "cuda")
        self.n_ch, self.n_t = int(n_ch), int(n_t)
        h = ctypes.c_void_p()
        idx = self.device.index if self.device.index is not None else torch.cuda.current_device()
        _check(lib().lps_data_create(self.n_ch, self.n_t, idx, ctypes.byref(h)), "lps_data_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _release("lps_data_destroy", self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def periodogram(self, x: torch.Tensor, dt, window=None, xyz_to_aet=False, out=None, stream=None):
        """P [n_ch, n_t//2 + 1] of device series x [n_ch, n_t] (contiguous FP64); out, if
        given, must be a contiguous FP64 tensor of that shape on the same device."""
        assert x.is_cuda and x.dtype == torch.float64 and x.is_contiguous() and tuple(x.shape) == (self.n_ch, self.n_t)
        assert window is None or (window.is_cuda and window.dtype == torch.float64 and window.is_contiguous())
        nf = self.n_t // 2 + 1
        P = out if out is not None else torch.empty((self.n_ch, nf), dtype=torch.float64, device=x.device)
        _check(lib().lps_data_periodogram_planned(self._h, _ptr(x), float(dt), _ptr(window), 1 if xyz_to_aet else 0,
                                                  _ptr(P), _stream(stream)), "lps_data_periodogram_planned")
        return P


def data_average(f: torch.Tensor, P: torch.Tensor, k0, seg_len, n_seg, stream=None):
    """Averaged periodogram over n_seg segments of seg_len bins from bin k0:
    returns (f_seg [n_seg], D [n_ch, n_seg], nu [n_seg]) on the device."""
    Pc = _dev(P, torch.float64, P.device)
    fc = _dev(f, torch.float64, P.device)
    n_ch, n_f = Pc.shape
    D = torch.empty((n_ch, n_seg), dtype=torch.float64, device=Pc.device)
    fs = torch.empty(n_seg, dtype=torch.float64, device=Pc.device)
    nu = torch.empty_like(fs)
    _check(lib().lps_data_average(_ptr(Pc), int(n_ch), int(n_f), _ptr(fc), int(k0), int(seg_len), int(n_seg),
                                  _ptr(D), _ptr(fs), _ptr(nu), _stream(stream)), "lps_data_average")
    return fs, D, nu


def data_response(grid_f, grid_R, f: torch.Tensor, stream=None):
    """Response grid_R [n_ch, n_g] at grid_f [n_g] interpolated to f (device):
    returns R [n_ch, len(f)] on the device."""
    fc = _dev(f, torch.float64, f.device)
    gf = _dev(grid_f, torch.float64, fc.device)
    gR = _dev(np.atleast_2d(grid_R) if not isinstance(grid_R, torch.Tensor) else grid_R, torch.float64, fc.device)
    n_ch, n_g = gR.shape
    R = torch.empty((n_ch, fc.numel()), dtype=torch.float64, device=fc.device)
    _check(lib().lps_data_response(_ptr(gf), _ptr(gR), int(n_ch), int(n_g), _ptr(fc), int(fc.numel()), _ptr(R),
                                   _stream(stream)), "lps_data_response")
    return R


def paper_ladder():
    """Inverse temperatures of the 20-rung ladder of Sec. "MCMC setup" (increasing),
    from lps_paper_ladder."""
    out = np.empty(20, dtype=np.float64)
    _check(lib().lps_paper_ladder(out.ctypes.data), "lps_paper_ladder")
    return out


def column_median(x: torch.Tensor, stream=None):
    """Median of every row of x [m, n] (device FP64, contiguous), from lps_column_median:
    returns a device tensor [m]."""
    assert x.is_cuda and x.dtype == torch.float64 and x.dim() == 2
    xc = x.contiguous()
    m, n = xc.shape
    out = torch.empty(m, dtype=torch.float64, device=xc.device)
    _check(lib().lps_column_median(_ptr(xc), int(n), int(m), int(n), _ptr(out), _stream(stream)), "lps_column_median")
    return out


def stepping_stone(betas, logL: torch.Tensor, stream=None):
    """Eq. (ss) over logL records [n_rec, T, W] (device FP64): returns
    (log Z, Var(log Z), log r_k [T-1], Var(log r_k) [T-1]) as host values."""
    n_rec, T, W = logL.shape
    lg = _dev(logL, torch.float64, logL.device)
    b = _dev(betas, torch.float64, lg.device)
    out = torch.empty(2 + 2 * (T - 1), dtype=torch.float64, device=lg.device)
    _check(lib().lps_stepping_stone(_ptr(b), int(T), _ptr(lg), int(n_rec), int(W), _ptr(out), _stream(stream)),
           "lps_stepping_stone")
    o = out.cpu().numpy()
    return float(o[0]), float(o[1]), o[2:2 + T - 1], o[2 + T - 1:]


def dic(logL: torch.Tensor, logL_at_mean, rung=-1, stream=None):
    """DIC over the draws of one rung of logL records [n_rec, T, W] (device FP64),
    with logL_at_mean = logL at the posterior-mean parameters: returns
    (mean D, p_D, DIC, Var D)."""
    n_rec, T, W = logL.shape
    lg = _dev(logL, torch.float64, logL.device)
    lm = _dev(np.array([float(logL_at_mean)]), torch.float64, lg.device)
    out = torch.empty(4, dtype=torch.float64, device=lg.device)
    _check(lib().lps_dic(_ptr(lg), int(n_rec), int(T), int(W), int(rung % T), _ptr(lm), _ptr(out), _stream(stream)),
           "lps_dic")
    return tuple(float(v) for v in out.cpu().numpy())


class Sampler:
    """Parallel-tempered reversible-jump sweeps on the device (wraps lps_sampler_*)."""

    KINDS = ("langevin", "birth", "death", "swap", "stretch")

    def __init__(self, ctx: Context, n_walkers, betas, seed=1, k_in_max=10, step=0.05, precision="mixed",
                 temp_scales=None, fixed_params=(), rj_moves=True, stretch_moves=False):
        _drain()
        self.ctx = ctx
        self.W = int(n_walkers)
        self.betas = np.ascontiguousarray(betas, dtype=np.float64)
        self.T = int(self.betas.size)
        self.C = self.W * self.T
        self.KC = int(k_in_max) + 2
        self._scales = None if temp_scales is None else np.ascontiguousarray(temp_scales, dtype=np.float64)
        d = _SamplerDesc()
        d.n_walkers, d.n_temps = self.W, self.T
        d.betas = self.betas.ctypes.data
        d.temp_scales = None if self._scales is None else self._scales.ctypes.data
        d.seed = int(seed)
        d.k_in_max = int(k_in_max)
        d.step = float(step)
        d.precision = _PREC.get(precision, precision)
        d.fixed_params = sum(1 << int(p) for p in fixed_params)
        d.rj_moves = 1 if rj_moves else 0
        d.stretch_moves = 1 if stretch_moves else 0
        h = ctypes.c_void_p()
        _check(lib().lps_sampler_create(ctx._h, ctypes.byref(d), ctypes.byref(h)), "lps_sampler_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _release("lps_sampler_destroy", self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, st: States, sweep_index=0, stream=None):
        c = st._c()
        _check(lib().lps_sampler_set_state(self._h, ctypes.byref(c), ctypes.c_uint64(int(sweep_index)),
                                           _stream(stream)), "lps_sampler_set_state")

    def sweep(self, n=1, stream=None):
        _check(lib().lps_sampler_sweep(self._h, int(n), _stream(stream)), "lps_sampler_sweep")

    def get_state(self, stream=None, sweep_index=True):
        dev, C, NS, KC = self.ctx.device, self.C, self.ctx.n_spl, self.KC
        params = torch.empty((self.ctx.n_params, C), dtype=torch.float64, device=dev)
        off = torch.empty(C * NS, dtype=torch.int32, device=dev)
        cnt = torch.empty(C * NS, dtype=torch.int32, device=dev)
        kx = torch.empty(C * NS * KC, dtype=torch.float64, device=dev)
        ky = torch.empty_like(kx)
        logL = torch.empty(C, dtype=torch.float64, device=dev)
        sw = ctypes.c_uint64()
        _check(lib().lps_sampler_get_state(self._h, _ptr(params), _ptr(off), _ptr(cnt), _ptr(kx), _ptr(ky),
                                           _ptr(logL), ctypes.byref(sw) if sweep_index else None, _stream(stream)),
               "lps_sampler_get_state")
        return {"params": params, "knot_off": off, "knot_cnt": cnt, "knot_x": kx, "knot_y": ky, "logL": logL,
                "sweep": sw.value if sweep_index else None}

    def record_logL(self, out_row: torch.Tensor, stream=None):
        """Copy the chains' current logL [T*W] into out_row (device FP64, e.g. a row
        of a [n_rec, T, W] record buffer); asynchronous, graph-capturable."""
        assert out_row.dtype == torch.float64 and out_row.numel() == self.C and out_row.is_contiguous()
        _check(lib().lps_sampler_get_state(self._h, None, None, None, None, None, _ptr(out_row), None,
                                           _stream(stream)), "lps_sampler_get_state")

    def packed_state(self, stream=None):
        """Current chains as a packed-CSR States batch (for checkpoints and set_state)."""
        s = self.get_state(stream)
        off, cnt = s["knot_off"].cpu().numpy(), s["knot_cnt"].cpu().numpy()
        kx, ky = s["knot_x"].cpu().numpy(), s["knot_y"].cpu().numpy()
        xs = [kx[o:o + c] for o, c in zip(off, cnt)]
        ys = [ky[o:o + c] for o, c in zip(off, cnt)]
        poff = np.zeros(len(cnt) + 1, dtype=np.int32)
        poff[1:] = np.cumsum(cnt)
        st = self.ctx.states(s["params"], poff, np.concatenate(xs), np.concatenate(ys))
        return st, s["sweep"], s["logL"]

    def counters(self, stream=None):
        k = len(self.KINDS)
        buf = (ctypes.c_uint32 * (k * self.T * 2))()
        _check(lib().lps_sampler_counters(self._h, buf, _stream(stream)), "lps_sampler_counters")
        return np.frombuffer(buf, dtype=np.uint32).reshape(k, self.T, 2).copy()


class LogLikeFn(torch.autograd.Function):
    """logL(theta) with the library's adjoint as its backward.

    forward(ctx_obj, precision, params, knot_x, knot_y, knot_off) -> logL [n]
    Gradients flow to params, knot_x and knot_y.
    """

    @staticmethod
    def forward(fctx, lctx: Context, precision, params, knot_x, knot_y, knot_off):
        st = States(params.detach().contiguous(), knot_off.contiguous(), knot_x.detach().contiguous(),
                    knot_y.detach().contiguous())
        logL, dp, dkx, dky, _ = lctx.loglike_grad_batch(st, precision)
        fctx.save_for_backward(dp, dkx, dky, knot_off)
        fctx.n_spl = lctx.n_spl
        return logL

    @staticmethod
    def backward(fctx, gout):
        dp, dkx, dky, knot_off = fctx.saved_tensors
        n = dp.shape[1]
        n_spl = fctx.n_spl
        if n_spl == 0:
            return None, None, dp * gout[None, :], None, None, None
        # owner state of every knot: knot i belongs to the state whose first slot
        # offset is the last one <= i (offsets relative to knot_off[0])
        first = (knot_off[0:n * n_spl:n_spl] - knot_off[0]).to(torch.int64)
        idx = torch.arange(dkx.numel(), device=dp.device, dtype=torch.int64)
        owner = torch.searchsorted(first, idx, right=True) - 1
        g_knot = gout[owner.clamp(min=0)]
        return None, None, dp * gout[None, :], dkx * g_knot, dky * g_knot, None
