"""Python binding of the F-chi2 C ABI (include/fchi2.h).

Argument marshalling only: every step of the search and of its adjoint runs in
the HIP kernels of libfchi2.so.  PyTorch supplies device memory and the
current stream.  The library must be built (``python -m
paper_0901_1913_amd.build``); nothing here falls back to another
implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfchi2.so")

OK, ERR_ARG, ERR_NOMEM, ERR_HIP, ERR_STATE, ERR_UNSUPPORTED = range(6)
FP64, MIXED = 0, 1
KEEP_FOR_BACKWARD, GRAPH, FUSED_SPREAD, WIDE_SOLVE, PERSISTENT, TWO_STREAMS = 1, 2, 4, 8, 16, 32
NOALLOC_SCRATCH_BYTES = 64 << 20
H_MAX = 16
H_MAX_REGISTER = 8
BIN_PIVOT, BIN_LOW_F, BIN_DC = 1, 2, 4
CURVE_NONFINITE, CURVE_UNSORTED, CURVE_WRAP, CURVE_FEW, CURVE_EMPTY = 8, 16, 32, 64, 128

EXPORTS = (
    "fchi2_plan", "fchi2_workspace_bytes", "fchi2_total_points", "fchi2_search",
    "fchi2_search_curves",
    "fchi2_backward", "fchi2_top_peaks_scratch_bytes", "fchi2_top_peaks",
    "fchi2_destroy", "fchi2_status_string", "fchi2_last_error", "fchi2_profile",
    "fchi2_profile_read", "fchi2_autotune", "fchi2_plan_info",
    "fchi2_search_top_workspace_bytes", "fchi2_search_top",
    "fchi2_fine_scratch_bytes", "fchi2_fine_search",
    "fchi2_search_multi_workspace_bytes", "fchi2_search_multi", "fchi2_detrend",
    "fchi2_autotune_multi", "fchi2_search_generation", "fchi2_backward_at",
    "fchi2_auto_n_freq", "fchi2_plan_n_freq", "fchi2_search_noalloc", "fchi2_search_coeffs",
    "fchi2_plan_set_schedule",
)
PROF_STAGES = ("moments", "spread", "fft_first", "fft_mid", "fft_last", "solve",
               "bwd_solve", "bwd_fft", "bwd_gather", "bwd_final", "top_merge",
               "fine", "persistent")


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("n_curves", ctypes.c_int32),
        ("offsets", ctypes.POINTER(ctypes.c_int64)),
        ("f_max", ctypes.c_double),
        ("H", ctypes.c_int32),
        ("n_freq", ctypes.c_int64),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("kernel_width", ctypes.c_int32),
        ("curves_per_wave", ctypes.c_int32),
        ("first_bin", ctypes.c_int64),
        ("oversampling", ctypes.c_double),
        ("t_span", ctypes.POINTER(ctypes.c_double)),
    ]


class TopOut(ctypes.Structure):
    _fields_ = [
        ("idx", ctypes.c_void_p),
        ("log_p", ctypes.c_void_p),
        ("dchi2", ctypes.c_void_p),
        ("dchi2_adj", ctypes.c_void_p),
        ("flags", ctypes.c_void_p),
        ("chi2_best", ctypes.c_void_p),
        ("curve_flags", ctypes.c_void_p),
    ]


class FineOut(ctypes.Structure):
    _fields_ = [
        ("rows", ctypes.c_void_p),
        ("f_best", ctypes.c_void_p),
        ("dchi2_best", ctypes.c_void_p),
        ("coef", ctypes.c_void_p),
        ("flags", ctypes.c_void_p),
    ]


class FChi2Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fchi2 status {status}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libfchi2.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_0901_1913_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64
    L.fchi2_plan.argtypes = [ctypes.POINTER(PlanDesc), vp, ctypes.POINTER(vp)]
    L.fchi2_plan.restype = ctypes.c_int
    L.fchi2_auto_n_freq.argtypes = [i32, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    L.fchi2_auto_n_freq.restype = i64
    L.fchi2_plan_n_freq.argtypes = [vp]
    L.fchi2_plan_n_freq.restype = i64
    L.fchi2_workspace_bytes.argtypes = [vp]
    L.fchi2_workspace_bytes.restype = sz
    L.fchi2_total_points.argtypes = [vp]
    L.fchi2_total_points.restype = i64
    L.fchi2_search.argtypes = [vp, vp, vp, vp, vp, sz, vp, vp, vp, vp]
    L.fchi2_search.restype = ctypes.c_int
    L.fchi2_search_coeffs.argtypes = [vp, vp, vp, vp, vp, sz, vp, vp, vp, vp, vp]
    L.fchi2_search_coeffs.restype = ctypes.c_int
    L.fchi2_search_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.fchi2_search_noalloc.restype = ctypes.c_int
    L.fchi2_search_curves.argtypes = [vp, i32, i32, vp, vp, vp, vp, sz, vp, vp, vp, vp]
    L.fchi2_search_curves.restype = ctypes.c_int
    L.fchi2_backward.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp, vp, vp]
    L.fchi2_backward.restype = ctypes.c_int
    L.fchi2_backward_at.argtypes = [vp, ctypes.c_uint64, vp, vp, vp, vp, vp, sz, vp, vp, vp]
    L.fchi2_backward_at.restype = ctypes.c_int
    L.fchi2_search_generation.argtypes = [vp]
    L.fchi2_search_generation.restype = ctypes.c_uint64
    L.fchi2_top_peaks_scratch_bytes.argtypes = [vp, i32]
    L.fchi2_top_peaks_scratch_bytes.restype = sz
    L.fchi2_top_peaks.argtypes = [vp, vp, i32, i64, i32, vp, sz, vp, vp]
    L.fchi2_top_peaks.restype = ctypes.c_int
    L.fchi2_destroy.argtypes = [vp]
    L.fchi2_destroy.restype = None
    L.fchi2_status_string.argtypes = [ctypes.c_int]
    L.fchi2_status_string.restype = ctypes.c_char_p
    L.fchi2_last_error.argtypes = []
    L.fchi2_last_error.restype = ctypes.c_char_p
    L.fchi2_profile.argtypes = [vp, i32]
    L.fchi2_profile.restype = ctypes.c_int
    L.fchi2_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64)]
    L.fchi2_profile_read.restype = ctypes.c_int
    L.fchi2_autotune.argtypes = [vp, vp, vp, vp, vp, sz, vp, ctypes.c_char_p, vp]
    L.fchi2_autotune.restype = ctypes.c_int
    L.fchi2_plan_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), i32]
    L.fchi2_plan_info.restype = ctypes.c_int
    L.fchi2_plan_set_schedule.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), i32]
    L.fchi2_plan_set_schedule.restype = ctypes.c_int
    L.fchi2_search_top_workspace_bytes.argtypes = [vp, i32]
    L.fchi2_search_top_workspace_bytes.restype = sz
    L.fchi2_search_top.argtypes = [vp, vp, vp, vp, vp, sz, i32, i64, i32, vp,
                                   ctypes.POINTER(TopOut), vp]
    L.fchi2_search_top.restype = ctypes.c_int
    L.fchi2_fine_scratch_bytes.argtypes = [vp, i32, i32]
    L.fchi2_fine_scratch_bytes.restype = sz
    L.fchi2_fine_search.argtypes = [vp, vp, vp, vp, vp, i32, i32, ctypes.c_double, i32, vp, sz,
                                    ctypes.POINTER(FineOut), vp]
    L.fchi2_fine_search.restype = ctypes.c_int
    L.fchi2_search_multi_workspace_bytes.argtypes = [vp, i32]
    L.fchi2_search_multi_workspace_bytes.restype = sz
    L.fchi2_search_multi.argtypes = [vp, vp, vp, vp, vp, i32, vp, sz, vp, vp, vp, vp]
    L.fchi2_search_multi.restype = ctypes.c_int
    L.fchi2_autotune_multi.argtypes = [vp, vp, vp, vp, vp, i32, vp, sz, vp, vp]
    L.fchi2_autotune_multi.restype = ctypes.c_int
    L.fchi2_detrend.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp]
    L.fchi2_detrend.restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != OK:
        msg = lib().fchi2_last_error().decode() or lib().fchi2_status_string(status).decode()
        raise FChi2Error(status, msg)


def _torch():
    import torch
    return torch


def _stream_handle(stream) -> int:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _dev_ptr(tensor, dtype, n=None, name="tensor"):
    torch = _torch()
    if not isinstance(tensor, torch.Tensor) or not tensor.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if tensor.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {tensor.dtype}")
    if not tensor.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and tensor.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {tensor.numel()}")
    return ctypes.c_void_p(tensor.data_ptr())


class Plan:
    """A search plan: geometry, FFT split and device tables for a set of curves.

    n_freq = 0 derives the grid from the spans (t_span, one per curve) and the
    oversampling factor (default 5) by the rule of auto_n_freq.

    first_bin = k0 > 0 makes a band plan: its rows hold bins k0 .. k0 + n_freq - 1
    of the search with bin spacing f_max / n_freq (one share of a search split by
    frequency band); such plans support search, search_curves and autotune."""

    def __init__(self, offsets: Sequence[int], f_max: float, H: int, n_freq: int,
                 precision: str = "mixed", keep_for_backward: bool = False,
                 graph: bool = False, kernel_width: int = 0, curves_per_wave: int = 0,
                 first_bin: int = 0, oversampling: float = 0.0, t_span=None,
                 fused_spread: bool = False, wide_solve: bool = False,
                 persistent: bool = False, two_streams: bool = False, stream=None):
        torch = _torch()
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        if off.ndim != 1 or off.shape[0] < 2:
            raise ValueError("offsets must be a 1-D array of n_curves + 1 entries")
        if precision not in ("mixed", "fp64"):
            raise ValueError("precision must be 'mixed' or 'fp64'")
        self._off = off
        flags = ((KEEP_FOR_BACKWARD if keep_for_backward else 0) | (GRAPH if graph else 0)
                 | (FUSED_SPREAD if fused_spread else 0) | (WIDE_SOLVE if wide_solve else 0)
                 | (PERSISTENT if persistent else 0) | (TWO_STREAMS if two_streams else 0))
        desc = PlanDesc(
            n_curves=off.shape[0] - 1,
            offsets=off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            f_max=float(f_max), H=int(H), n_freq=int(n_freq),
            precision=FP64 if precision == "fp64" else MIXED,
            flags=flags, kernel_width=int(kernel_width), first_bin=int(first_bin),
            curves_per_wave=int(curves_per_wave), oversampling=float(oversampling))
        if t_span is not None:
            spans = np.ascontiguousarray(np.asarray(t_span, dtype=np.float64))
            if spans.shape != (off.shape[0] - 1,):
                raise ValueError("t_span must hold one span per curve")
            desc.t_span = spans.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        handle = ctypes.c_void_p()
        st = _stream_handle(stream) if torch.cuda.is_available() else 0
        _check(lib().fchi2_plan(ctypes.byref(desc), ctypes.c_void_p(st), ctypes.byref(handle)))
        self._h = handle
        self.offsets = off.copy()
        self.n_curves = off.shape[0] - 1
        self.n_total = int(off[-1])
        self.H, self.f_max = int(H), float(f_max)
        self.n_freq = int(lib().fchi2_plan_n_freq(self._h))
        self.precision = precision
        self.first_bin = int(first_bin)
        self.keep_for_backward = keep_for_backward
        self.out_dtype = torch.float64 if precision == "fp64" else torch.float32
        self.workspace_bytes = int(lib().fchi2_workspace_bytes(self._h))
        self._ws = None

    # -- memory -----------------------------------------------------------
    def workspace(self, device="cuda", nbytes: int = 0):
        """Allocate and return the plan's workspace tensor (grown to nbytes if needed;
        growing discards the state a later backward() needs)."""
        torch = _torch()
        need = max(self.workspace_bytes, int(nbytes), 256)
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            # torch allocations are 512-byte aligned on ROCm.
            self._ws = torch.empty(need, dtype=torch.uint8, device=device)
        return self._ws

    @property
    def freqs(self) -> np.ndarray:
        return np.arange(self.n_freq, dtype=np.float64) * (self.f_max / self.n_freq)

    # -- entry points ---------------------------------------------------------
    def search(self, t, x, sigma, dchi2=None, chi2_0=None, flags=None, workspace=None,
               stream=None, want_flags=True):
        """Delta chi2 [n_curves, H, n_freq], chi2_0 [n_curves], flags [n_curves, n_freq]."""
        torch = _torch()
        f64 = torch.float64
        pt = _dev_ptr(t, f64, self.n_total, "t")
        px = _dev_ptr(x, f64, self.n_total, "x")
        ps = _dev_ptr(sigma, f64, self.n_total, "sigma")
        dev = t.device
        if dchi2 is None:
            dchi2 = torch.empty((self.n_curves, self.H, self.n_freq), dtype=self.out_dtype,
                                device=dev)
        if chi2_0 is None:
            chi2_0 = torch.empty(self.n_curves, dtype=f64, device=dev)
        if flags is None and want_flags:
            flags = torch.empty((self.n_curves, self.n_freq), dtype=torch.uint8, device=dev)
        ws = self.workspace(dev) if workspace is None else workspace
        _check(lib().fchi2_search(
            self._h, pt, px, ps, ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
            _dev_ptr(dchi2, self.out_dtype, self.n_curves * self.H * self.n_freq, "dchi2"),
            _dev_ptr(chi2_0, f64, self.n_curves, "chi2_0"),
            _dev_ptr(flags, torch.uint8, self.n_curves * self.n_freq, "flags")
            if flags is not None else ctypes.c_void_p(0),
            ctypes.c_void_p(_stream_handle(stream))))
        return dchi2, chi2_0, flags

    def search_coeffs(self, t, x, sigma, workspace=None, stream=None):
        """Delta chi2, chi2_0, flags and the H model's coefficients
        [n_curves, 2H+1, n_freq] (xbar added to A_0; basis in t - first time)."""
        torch = _torch()
        f64 = torch.float64
        dev = t.device
        nc, H, nf = self.n_curves, self.H, self.n_freq
        dchi2 = torch.empty((nc, H, nf), dtype=self.out_dtype, device=dev)
        chi2_0 = torch.empty(nc, dtype=f64, device=dev)
        flags = torch.empty((nc, nf), dtype=torch.uint8, device=dev)
        coef = torch.empty((nc, 2 * H + 1, nf), dtype=self.out_dtype, device=dev)
        ws = self.workspace(dev) if workspace is None else workspace
        _check(lib().fchi2_search_coeffs(
            self._h, _dev_ptr(t, f64, self.n_total, "t"), _dev_ptr(x, f64, self.n_total, "x"),
            _dev_ptr(sigma, f64, self.n_total, "sigma"), ctypes.c_void_p(ws.data_ptr()),
            ctypes.c_size_t(ws.numel()), ctypes.c_void_p(dchi2.data_ptr()),
            ctypes.c_void_p(chi2_0.data_ptr()), ctypes.c_void_p(flags.data_ptr()),
            ctypes.c_void_p(coef.data_ptr()), ctypes.c_void_p(_stream_handle(stream))))
        return dchi2, chi2_0, flags, coef

    def search_noalloc(self, t, x, sigma, dchi2, chi2_0, flags=None, stream=None):
        """fchi2_search into caller outputs with the library's device scratch as
        workspace (no allocation); the plan's workspace must fit in
        NOALLOC_SCRATCH_BYTES."""
        torch = _torch()
        f64 = torch.float64
        _check(lib().fchi2_search_noalloc(
            self._h, _dev_ptr(t, f64, self.n_total, "t"), _dev_ptr(x, f64, self.n_total, "x"),
            _dev_ptr(sigma, f64, self.n_total, "sigma"),
            _dev_ptr(dchi2, self.out_dtype, self.n_curves * self.H * self.n_freq, "dchi2"),
            _dev_ptr(chi2_0, f64, self.n_curves, "chi2_0"),
            _dev_ptr(flags, torch.uint8, self.n_curves * self.n_freq, "flags")
            if flags is not None else ctypes.c_void_p(0),
            ctypes.c_void_p(_stream_handle(stream))))
        return dchi2, chi2_0, flags

    def search_curves(self, first: int, count: int, t, x, sigma, dchi2, chi2_0, flags=None,
                      workspace=None, stream=None):
        """fchi2_search on curves [first, first + count) into full-size outputs."""
        torch = _torch()
        f64 = torch.float64
        ws = self.workspace(t.device) if workspace is None else workspace
        _check(lib().fchi2_search_curves(
            self._h, int(first), int(count), _dev_ptr(t, f64, self.n_total, "t"),
            _dev_ptr(x, f64, self.n_total, "x"), _dev_ptr(sigma, f64, self.n_total, "sigma"),
            ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
            _dev_ptr(dchi2, self.out_dtype, self.n_curves * self.H * self.n_freq, "dchi2"),
            _dev_ptr(chi2_0, f64, self.n_curves, "chi2_0"),
            _dev_ptr(flags, torch.uint8, self.n_curves * self.n_freq, "flags")
            if flags is not None else ctypes.c_void_p(0),
            ctypes.c_void_p(_stream_handle(stream))))
        return dchi2, chi2_0, flags

    def search_top(self, t, x, sigma, K: int = 16, hrow: Optional[int] = None, k_lo: int = 0,
                   workspace=None, stream=None):
        """Search with the significance epilogue: per curve the K bins of smallest
        ln p = ln k + ln Q(Delta chi2 | 2H') among the local maxima of row hrow.

        Returns a dict of device tensors: idx [n_curves, K] int64 (-1 past the
        last candidate), log_p [n_curves, K], dchi2 [n_curves, K, H],
        dchi2_adj [n_curves, K], flags [n_curves, K] uint8, chi2_best and
        chi2_0 [n_curves], curve_flags [n_curves] uint8.
        """
        torch = _torch()
        f64 = torch.float64
        hrow = self.H - 1 if hrow is None else int(hrow)
        dev = t.device
        nc = self.n_curves
        res = {
            "idx": torch.empty((nc, K), dtype=torch.int64, device=dev),
            "log_p": torch.empty((nc, K), dtype=f64, device=dev),
            "dchi2": torch.empty((nc, K, self.H), dtype=f64, device=dev),
            "dchi2_adj": torch.empty((nc, K), dtype=f64, device=dev),
            "flags": torch.empty((nc, K), dtype=torch.uint8, device=dev),
            "chi2_best": torch.empty(nc, dtype=f64, device=dev),
            "chi2_0": torch.empty(nc, dtype=f64, device=dev),
            "curve_flags": torch.empty(nc, dtype=torch.uint8, device=dev),
        }
        need = int(lib().fchi2_search_top_workspace_bytes(self._h, int(K)))
        if need == 0:
            raise FChi2Error(ERR_ARG, "K must be in 1..64")
        ws = self.workspace(dev, need) if workspace is None else workspace
        out = TopOut(*(ctypes.c_void_p(res[k].data_ptr()) for k in
                       ("idx", "log_p", "dchi2", "dchi2_adj", "flags", "chi2_best",
                        "curve_flags")))
        _check(lib().fchi2_search_top(
            self._h, _dev_ptr(t, f64, self.n_total, "t"), _dev_ptr(x, f64, self.n_total, "x"),
            _dev_ptr(sigma, f64, self.n_total, "sigma"), ctypes.c_void_p(ws.data_ptr()),
            ctypes.c_size_t(ws.numel()), int(hrow), int(k_lo), int(K),
            ctypes.c_void_p(res["chi2_0"].data_ptr()), ctypes.byref(out),
            ctypes.c_void_p(_stream_handle(stream))))
        return res

    def detrend(self, t, x, sigma, degree: int, x_out=None, want_coef=False, stream=None):
        """Residuals of each curve's weighted least-squares polynomial fit
        (degree 0..3); returns x_out (and the Legendre coefficients)."""
        torch = _torch()
        f64 = torch.float64
        if x_out is None:
            x_out = torch.empty_like(x)
        coef = (torch.empty((self.n_curves, int(degree) + 1), dtype=f64, device=t.device)
                if want_coef else None)
        _check(lib().fchi2_detrend(
            self._h, _dev_ptr(t, f64, self.n_total, "t"), _dev_ptr(x, f64, self.n_total, "x"),
            _dev_ptr(sigma, f64, self.n_total, "sigma"), int(degree),
            _dev_ptr(x_out, f64, self.n_total, "x_out"),
            _dev_ptr(coef, f64, None, "coef") if coef is not None else ctypes.c_void_p(0),
            ctypes.c_void_p(_stream_handle(stream))))
        return (x_out, coef) if want_coef else x_out

    def autotune_multi(self, t, sigma, x, scale, stream=None):
        """Pick the FFT split and spreading tile for search_multi on these data."""
        torch = _torch()
        f64 = torch.float64
        S = int(x.shape[0])
        nbytes = int(lib().fchi2_search_multi_workspace_bytes(self._h, S))
        if nbytes == 0:
            raise FChi2Error(ERR_UNSUPPORTED, "shared-alpha search needs a plan of one curve, "
                             "H <= 5 and no band (first_bin = 0)")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=t.device)
        scratch = torch.empty((S, self.H, self.n_freq), dtype=self.out_dtype, device=t.device)
        _check(lib().fchi2_autotune_multi(
            self._h, _dev_ptr(t, f64, self.n_total, "t"),
            _dev_ptr(sigma, f64, self.n_total, "sigma"), _dev_ptr(x, f64, S * self.n_total, "x"),
            _dev_ptr(scale, f64, S, "scale"), S, ctypes.c_void_p(ws.data_ptr()),
            ctypes.c_size_t(nbytes), ctypes.c_void_p(scratch.data_ptr()),
            ctypes.c_void_p(_stream_handle(stream))))
        return self.info()

    def search_multi(self, t, sigma, x, scale, want_flags=True, stream=None):
        """Shared-alpha search of sources observed at the plan's single time base.

        t, sigma: device FP64 [n]; x: device FP64 [n_sources, n]; scale: device
        FP64 [n_sources] (source errors are scale * sigma).  Returns
        (dchi2 [n_sources, H, n_freq], chi2_0 [n_sources], flags [n_freq]).
        """
        torch = _torch()
        f64 = torch.float64
        if self.n_curves != 1:
            raise ValueError("search_multi needs a plan of one curve (the shared time base)")
        if x.dim() != 2 or x.shape[1] != self.n_total:
            raise ValueError("x must have shape [n_sources, n]")
        S = int(x.shape[0])
        dev = t.device
        nbytes = int(lib().fchi2_search_multi_workspace_bytes(self._h, S))
        if nbytes == 0:
            raise FChi2Error(ERR_UNSUPPORTED, "shared-alpha search needs a plan of one curve, "
                             "H <= 5 and no band (first_bin = 0)")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        dchi2 = torch.empty((S, self.H, self.n_freq), dtype=self.out_dtype, device=dev)
        chi2_0 = torch.empty(S, dtype=f64, device=dev)
        flags = torch.empty(self.n_freq, dtype=torch.uint8, device=dev) if want_flags else None
        _check(lib().fchi2_search_multi(
            self._h, _dev_ptr(t, f64, self.n_total, "t"),
            _dev_ptr(sigma, f64, self.n_total, "sigma"), _dev_ptr(x, f64, S * self.n_total, "x"),
            _dev_ptr(scale, f64, S, "scale"), S, ctypes.c_void_p(ws.data_ptr()),
            ctypes.c_size_t(nbytes),
            _dev_ptr(dchi2, self.out_dtype, S * self.H * self.n_freq, "dchi2"),
            _dev_ptr(chi2_0, f64, S, "chi2_0"),
            _dev_ptr(flags, torch.uint8, self.n_freq, "flags") if flags is not None
            else ctypes.c_void_p(0), ctypes.c_void_p(_stream_handle(stream))))
        return dchi2, chi2_0, flags

    def fine_search(self, t, x, sigma, f_center, R: int = 64,
                    half_width: Optional[float] = None, hrow: Optional[int] = None,
                    want_rows: bool = False, stream=None):
        """Direct (ungridded) Delta chi2 at R trial frequencies around each centre.

        f_center: device FP64 [n_curves, K] (NaN for none).  half_width defaults
        to one grid step f_max / n_freq.  Returns a dict of device tensors:
        f_best [n_curves, K], dchi2_best [n_curves, K, H], coef
        [n_curves, K, 2H+1] (xbar added to A_0; basis in t - first time),
        flags [n_curves, K] uint8 and, with want_rows, rows [n_curves, K, R, H].
        """
        torch = _torch()
        f64 = torch.float64
        if f_center.dim() != 2 or f_center.shape[0] != self.n_curves:
            raise ValueError("f_center must have shape [n_curves, K]")
        K = int(f_center.shape[1])
        hw = self.f_max / self.n_freq if half_width is None else float(half_width)
        hrow = self.H - 1 if hrow is None else int(hrow)
        dev = t.device
        nc, H = self.n_curves, self.H
        res = {
            "f_best": torch.empty((nc, K), dtype=f64, device=dev),
            "dchi2_best": torch.empty((nc, K, H), dtype=f64, device=dev),
            "coef": torch.empty((nc, K, 2 * H + 1), dtype=f64, device=dev),
            "flags": torch.empty((nc, K), dtype=torch.uint8, device=dev),
        }
        if want_rows:
            res["rows"] = torch.empty((nc, K, R, H), dtype=f64, device=dev)
        nbytes = int(lib().fchi2_fine_scratch_bytes(self._h, K, int(R)))
        if nbytes == 0:
            raise FChi2Error(ERR_ARG, "K must be in 1..256 and R in 1..4096")
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        out = FineOut(
            ctypes.c_void_p(res["rows"].data_ptr()) if want_rows else ctypes.c_void_p(0),
            ctypes.c_void_p(res["f_best"].data_ptr()),
            ctypes.c_void_p(res["dchi2_best"].data_ptr()),
            ctypes.c_void_p(res["coef"].data_ptr()), ctypes.c_void_p(res["flags"].data_ptr()))
        _check(lib().fchi2_fine_search(
            self._h, _dev_ptr(t, f64, self.n_total, "t"), _dev_ptr(x, f64, self.n_total, "x"),
            _dev_ptr(sigma, f64, self.n_total, "sigma"),
            _dev_ptr(f_center, f64, nc * K, "f_center"), K, int(R), hw, int(hrow),
            ctypes.c_void_p(scratch.data_ptr()), ctypes.c_size_t(nbytes), ctypes.byref(out),
            ctypes.c_void_p(_stream_handle(stream))))
        return res

    def refine(self, t, x, sigma, f_center, levels: int = 3, R: int = 64,
               hrow: Optional[int] = None, stream=None):
        """Zoom around each centre: level 1 spans +-1 grid step; each further
        level spans +-2 trial steps of the previous one around its best."""
        hw = self.f_max / self.n_freq
        res = None
        for _ in range(max(1, int(levels))):
            res = self.fine_search(t, x, sigma, f_center, R=R, half_width=hw, hrow=hrow,
                                   stream=stream)
            f_center = res["f_best"]
            hw = 2.0 * hw / max(R - 1, 1)
        return res

    def generation(self) -> int:
        """Number of searches run on the plan so far (see fchi2_search_generation)."""
        return int(lib().fchi2_search_generation(self._h))

    def backward(self, t, x, sigma, grad_dchi2, grad_x=None, grad_sigma=None,
                 workspace=None, stream=None, generation: Optional[int] = None):
        """dLoss/dx and dLoss/dsigma given dLoss/dDelta chi2 (same layout as dchi2).

        generation: the plan's generation right after the forward search to
        differentiate; if another search ran since, this raises (FCHI2_ERR_STATE)
        instead of differentiating the other search.  None: the last search."""
        torch = _torch()
        f64 = torch.float64
        dev = t.device
        if grad_x is None:
            grad_x = torch.empty(self.n_total, dtype=f64, device=dev)
        if grad_sigma is None:
            grad_sigma = torch.empty(self.n_total, dtype=f64, device=dev)
        ws = self.workspace(dev) if workspace is None else workspace
        gen = self.generation() if generation is None else int(generation)
        _check(lib().fchi2_backward_at(
            self._h, ctypes.c_uint64(gen), _dev_ptr(t, f64, self.n_total, "t"),
            _dev_ptr(x, f64, self.n_total, "x"),
            _dev_ptr(sigma, f64, self.n_total, "sigma"),
            _dev_ptr(grad_dchi2, self.out_dtype, self.n_curves * self.H * self.n_freq,
                     "grad_dchi2"),
            ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
            _dev_ptr(grad_x, f64, self.n_total, "grad_x"),
            _dev_ptr(grad_sigma, f64, self.n_total, "grad_sigma"),
            ctypes.c_void_p(_stream_handle(stream))))
        return grad_x, grad_sigma

    def top_peaks(self, dchi2, hrow: int, k_lo: int, K: int, out=None, stream=None):
        """[n_curves, K] int64 bins of the K largest strict local maxima (-1 if fewer)."""
        torch = _torch()
        nbytes = int(lib().fchi2_top_peaks_scratch_bytes(self._h, int(K)))
        scratch = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dchi2.device)
        if out is None:
            out = torch.empty((self.n_curves, K), dtype=torch.int64, device=dchi2.device)
        _check(lib().fchi2_top_peaks(
            self._h, _dev_ptr(dchi2, self.out_dtype, None, "dchi2"), int(hrow), int(k_lo),
            int(K), ctypes.c_void_p(scratch.data_ptr()), ctypes.c_size_t(scratch.numel()),
            _dev_ptr(out, torch.int64, self.n_curves * K, "out"),
            ctypes.c_void_p(_stream_handle(stream))))
        return out

    def autotune(self, t, x, sigma, cache_path: Optional[str] = None, workspace=None,
                 stream=None):
        """Time the candidate schedules on these inputs and keep the fastest."""
        torch = _torch()
        f64 = torch.float64
        ws = self.workspace(t.device) if workspace is None else workspace
        scratch = torch.empty((self.n_curves, self.H, self.n_freq), dtype=self.out_dtype,
                              device=t.device)
        _check(lib().fchi2_autotune(
            self._h, _dev_ptr(t, f64, self.n_total, "t"), _dev_ptr(x, f64, self.n_total, "x"),
            _dev_ptr(sigma, f64, self.n_total, "sigma"), ctypes.c_void_p(ws.data_ptr()),
            ctypes.c_size_t(ws.numel()), ctypes.c_void_p(scratch.data_ptr()),
            cache_path.encode() if cache_path else None,
            ctypes.c_void_p(_stream_handle(stream))))
        return self.info()

    def info(self) -> dict:
        """The plan's schedule: FFT radices, spreading tile, wave, kernel width."""
        arr = (ctypes.c_int32 * 15)()
        _check(lib().fchi2_plan_info(self._h, arr, 15))
        np_ = int(arr[0])
        return {"fft_log_radices": [int(arr[q]) for q in range(1, np_ + 1)],
                "fft_log_tiles": [int(arr[7 + q]) for q in range(1, np_ + 1)],
                "spread_tile": 1 << int(arr[5]), "curves_per_wave": int(arr[6]),
                "kernel_width": int(arr[7]), "fused_spread": bool(arr[12]),
                "persistent": bool(arr[13]), "solve_sub_wave": int(arr[14])}

    def set_schedule(self, schedule: dict) -> dict:
        """Apply a schedule as info() reports it (FFT radices and tiles,
        spreading tile, curves per wave, fused, persistent) without timing."""
        arr = (ctypes.c_int32 * 15)()
        ln = list(schedule["fft_log_radices"])
        le = list(schedule["fft_log_tiles"])
        if len(ln) != len(le) or not 1 <= len(ln) <= 4:
            raise ValueError("fft_log_radices and fft_log_tiles must have 1..4 equal entries")
        tile = int(schedule["spread_tile"])
        if tile <= 0 or tile & (tile - 1):
            raise ValueError("spread_tile must be a power of two")
        arr[0] = len(ln)
        for q, (a, b) in enumerate(zip(ln, le), 1):
            arr[q] = int(a)
            arr[7 + q] = int(b)
        arr[5] = tile.bit_length() - 1
        arr[6] = int(schedule["curves_per_wave"])
        arr[12] = 1 if schedule.get("fused_spread") else 0
        arr[13] = 1 if schedule.get("persistent") else 0
        arr[14] = int(schedule.get("solve_sub_wave", 0))
        _check(lib().fchi2_plan_set_schedule(self._h, arr, 15))
        return self.info()

    def profile(self, enable: bool = True):
        """Start (or stop) recording HIP event pairs around every launch."""
        _check(lib().fchi2_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """{stage: (total_ms, launches)} accumulated since profile() (waits for events)."""
        n = len(PROF_STAGES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(lib().fchi2_profile_read(self._h, ms, cnt))
        return {PROF_STAGES[i]: (float(ms[i]), int(cnt[i])) for i in range(n)}

    def close(self):
        if getattr(self, "_h", None):
            lib().fchi2_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def auto_n_freq(H: int, f_max: float, oversampling: float, span: float) -> int:
    """The plan's n_freq = 0 rule: next power of two >= ceil(os H span f_max),
    at least 2^10 (0 if out of range)."""
    return int(lib().fchi2_auto_n_freq(int(H), float(f_max), float(oversampling), float(span)))


def search(t, x, sigma, f_max: float, H: int, n_freq: int, precision: str = "mixed",
           offsets=None, **plan_kw):
    """One-shot search over device tensors; returns (dchi2, chi2_0, flags)."""
    if offsets is None:
        offsets = [0, int(t.numel())]
    plan = Plan(offsets, f_max, H, n_freq, precision=precision, **plan_kw)
    try:
        return plan.search(t, x, sigma)
    finally:
        import torch
        torch.cuda.current_stream().synchronize()
        plan.close()


def _make_autograd():
    torch = _torch()

    class FChi2Fn(torch.autograd.Function):
        """Delta chi2 with the hand-written adjoint as its backward.

        forward(t, x, sigma, plan, sort=False) -> dchi2 [n_curves, H, n_freq];
        the plan must have keep_for_backward=True.  With sort=True the points
        of each curve are first put in time order (the library itself flags
        an unsorted curve and gives it NaN rows), and the gradients are
        returned in the caller's order.  backward returns gradients for x and
        sigma (t is not differentiated).
        """

        @staticmethod
        def forward(ctx, t, x, sigma, plan, sort=False):
            if not plan.keep_for_backward:
                raise ValueError("FChi2Fn needs a plan with keep_for_backward=True")
            perm = None
            if sort:
                perm = time_order(plan.offsets, t)
                t, x, sigma = t[perm], x[perm], sigma[perm]
            dchi2, _, _ = plan.search(t, x, sigma, want_flags=False)
            ctx.plan = plan
            ctx.generation = plan.generation()
            ctx.perm = perm
            ctx.save_for_backward(t, x, sigma)
            return dchi2

        @staticmethod
        def backward(ctx, grad):
            t, x, sigma = ctx.saved_tensors
            plan = ctx.plan
            g = grad.to(plan.out_dtype).contiguous()
            gx, gs = plan.backward(t, x, sigma, g, generation=ctx.generation)
            if ctx.perm is not None:  # back to the caller's order
                ux, us = torch.empty_like(gx), torch.empty_like(gs)
                ux[ctx.perm] = gx
                us[ctx.perm] = gs
                gx, gs = ux, us
            return None, gx, gs, None, None

    return FChi2Fn


def time_order(offsets, t):
    """Device permutation that puts the points of each curve (CSR offsets) in
    ascending time, stably: t[perm] is sorted within every curve and the
    curves keep their ranges."""
    torch = _torch()
    off = torch.as_tensor(np.asarray(offsets, dtype=np.int64), device=t.device)
    counts = off[1:] - off[:-1]
    curve = torch.repeat_interleave(torch.arange(counts.numel(), device=t.device), counts)
    by_t = torch.argsort(t, stable=True)
    return by_t[torch.argsort(curve[by_t], stable=True)]


class _Lazy:
    _fn = None

    def __get__(self, obj, objtype=None):
        if _Lazy._fn is None:
            _Lazy._fn = _make_autograd()
        return _Lazy._fn


class _Holder:
    FChi2Fn = _Lazy()


def fchi2_fn():
    """The torch.autograd.Function wrapping search/backward."""
    return _Holder.FChi2Fn
