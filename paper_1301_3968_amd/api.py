"""Python face of libdedisp: plans over torch device tensors.

Only argument marshalling happens here; every step of the dedispersion and the
detection runs in the HIP library.  Device tensors must live on the current HIP
device; work is enqueued on torch's current stream.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L

_TORCH_DT = {torch.uint8: L.U8, torch.float32: L.F32, torch.int32: L.I32}


def _ptr(a) -> ctypes.c_void_p:
    if isinstance(a, torch.Tensor):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_check(t: torch.Tensor, name: str) -> None:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.stride(-1) != 1:
        raise ValueError(f"{name} must be contiguous along time")


class Plan:
    """Sample-set tables for a set of trial DMs (see include/dedisp.h).

    rule: 'smear' | 'allnonzero' | 'greedy' | 'explicit' | 'fixed'
    wmode: 'unit' | 'channel' | 'tap'
    """

    def __init__(self, freq_ghz, chan_bw_ghz: float, dt_s: float, dms, rule: str = "smear",
                 k_dm: float = 0.0, width_s: float = 0.0, scatter_s_1ghz: float = 0.0,
                 scatter_index: float = -4.0, spectral_index: float = 0.0, nu0_ghz: float = 0.0,
                 start=None, ntap=None, ktaps: int = 1, wmode: str = "unit", weights=None):
        lib = L.lib()
        self._freq = np.ascontiguousarray(freq_ghz, dtype=np.float64)
        self._dms = np.ascontiguousarray(dms, dtype=np.float64)
        prof = L.Profile()
        L.check(lib.dedisp_profile_init(ctypes.byref(prof)))
        prof.rule = L.RULES[rule]
        prof.k_dm = k_dm
        prof.width_s = width_s
        prof.scatter_s_1ghz = scatter_s_1ghz
        prof.scatter_index = scatter_index
        prof.spectral_index = spectral_index
        prof.nu0_ghz = nu0_ghz
        prof.ktaps = ktaps
        prof.wmode = L.WMODES[wmode]
        keep = []
        if start is not None:
            s = np.ascontiguousarray(start, dtype=np.int32)
            n = np.ascontiguousarray(ntap, dtype=np.int32)
            keep += [s, n]
            prof.start = s.ctypes.data
            prof.ntap = n.ctypes.data
        if weights is not None:
            w = np.ascontiguousarray(weights, dtype=np.float32)
            keep.append(w)
            prof.weights = w.ctypes.data
        h = ctypes.c_void_p()
        L.check(lib.dedisp_plan_create(ctypes.byref(h), len(self._freq), _ptr(self._freq),
                                       chan_bw_ghz, dt_s, len(self._dms), _ptr(self._dms),
                                       ctypes.byref(prof)))
        self._h = h
        self.nchan = len(self._freq)
        self.ndm = len(self._dms)
        self.wmode = wmode
        self.ktaps = ktaps if wmode == "tap" else 1
        info = [ctypes.c_int32() for _ in range(5)]
        L.check(lib.dedisp_plan_info(h, *[ctypes.byref(i) for i in info]))
        self.max_span = info[2].value

    def close(self) -> None:
        if getattr(self, "_h", None):
            L.lib().dedisp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def tables(self):
        s = np.empty((self.ndm, self.nchan), dtype=np.int32)
        n = np.empty((self.ndm, self.nchan), dtype=np.int32)
        L.check(L.lib().dedisp_plan_tables(self._h, _ptr(s), _ptr(n)))
        return s, n

    def out_len(self, nsamp: int) -> int:
        v = ctypes.c_int64()
        L.check(L.lib().dedisp_plan_out_len(self._h, nsamp, ctypes.byref(v)))
        return v.value

    def work_bytes(self, nsamp: int, nw: int) -> int:
        v = ctypes.c_size_t()
        L.check(L.lib().dedisp_work_bytes(self._h, nsamp, nw, ctypes.byref(v)))
        return v.value

    # ------------------------------------------------------------------ forward
    def dedisperse(self, x: torch.Tensor, out_dtype: Optional[torch.dtype] = None,
                   weights: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None):
        """y[(b,) d, t] for x[(b,) c, t] (uint8 or float32 device tensor)."""
        _dev_check(x, "x")
        xb = x if x.dim() == 3 else x.unsqueeze(0)
        B, C, T = xb.shape
        if C != self.nchan:
            raise ValueError("channel count differs from the plan")
        nout = self.out_len(T)
        if out_dtype is None:
            out_dtype = torch.int32 if (x.dtype == torch.uint8 and self.wmode == "unit") else torch.float32
        if out is None:
            out = torch.empty((B, self.ndm, nout), dtype=out_dtype, device=x.device)
        wptr = None
        if weights is not None:
            _dev_check(weights, "weights")
            weights = weights.contiguous().to(torch.float32)
            wptr = _ptr(weights)
        L.check(L.lib().dedisp_dedisperse(
            self._h, _ptr(xb), _TORCH_DT[x.dtype], T, xb.stride(1), xb.stride(0), B, _ptr(out),
            _TORCH_DT[out.dtype], out.stride(1), out.stride(0), wptr, _stream()))
        return out if x.dim() == 3 else out[0]

    def _widths(self, widths: Sequence[int]) -> np.ndarray:
        return np.ascontiguousarray(widths, dtype=np.int32)

    def _meansig(self, mean, sigma, device):
        m = torch.as_tensor(np.asarray(mean, dtype=np.float64), device=device)
        s = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)
        return m.contiguous(), s.contiguous()

    def detect(self, y: torch.Tensor, widths: Sequence[int], mean, sigma,
               work: Optional[torch.Tensor] = None):
        """Best boxcar (snr f64, t i32, W i32) per trial of a dedispersed block y[d, t]."""
        _dev_check(y, "y")
        D, nout = y.shape
        w = self._widths(widths)
        m, s = (mean, sigma) if isinstance(mean, torch.Tensor) else self._meansig(mean, sigma, y.device)
        need = self.work_bytes(nout + self.max_span - 1, len(w))
        if work is None or work.numel() < need:
            work = torch.empty(need, dtype=torch.uint8, device=y.device)
        snr = torch.empty(D, dtype=torch.float64, device=y.device)
        t = torch.empty(D, dtype=torch.int32, device=y.device)
        W = torch.empty(D, dtype=torch.int32, device=y.device)
        L.check(L.lib().dedisp_detect(self._h, _ptr(y), _TORCH_DT[y.dtype], nout, y.stride(0), _ptr(w),
                                      len(w), _ptr(m), _ptr(s), _ptr(snr), _ptr(t), _ptr(W),
                                      _ptr(work), work.numel(), _stream()))
        return snr, t, W

    def search(self, x: torch.Tensor, widths: Sequence[int], mean, sigma,
               work: Optional[torch.Tensor] = None, outputs=None):
        """Fused dedispersion + boxcar search of one block x[c, t]."""
        _dev_check(x, "x")
        C, T = x.shape
        w = self._widths(widths)
        m, s = (mean, sigma) if isinstance(mean, torch.Tensor) else self._meansig(mean, sigma, x.device)
        need = self.work_bytes(T, len(w))
        if work is None or work.numel() < need:
            work = torch.empty(need, dtype=torch.uint8, device=x.device)
        if outputs is None:
            outputs = (torch.empty(self.ndm, dtype=torch.float64, device=x.device),
                       torch.empty(self.ndm, dtype=torch.int32, device=x.device),
                       torch.empty(self.ndm, dtype=torch.int32, device=x.device))
        snr, t, W = outputs
        L.check(L.lib().dedisp_search(self._h, _ptr(x), _TORCH_DT[x.dtype], T, x.stride(0), _ptr(w),
                                      len(w), _ptr(m), _ptr(s), _ptr(snr), _ptr(t), _ptr(W),
                                      _ptr(work), work.numel(), _stream()))
        return snr, t, W

    def search_noalloc(self, x: torch.Tensor, widths: Sequence[int], mean: torch.Tensor,
                       sigma: torch.Tensor, outputs):
        """The fused search without a workspace (dedisp_search_noalloc): the library
        allocates nothing; mean, sigma are device fp64 [nchan] and outputs a
        preallocated device (snr f64, t i32, W i32) triple of [ndm] tensors."""
        _dev_check(x, "x")
        C, T = x.shape
        w = self._widths(widths)
        snr, t, W = outputs
        L.check(L.lib().dedisp_search_noalloc(self._h, _ptr(x), _TORCH_DT[x.dtype], T,
                                              x.stride(0), _ptr(w), len(w), _ptr(mean),
                                              _ptr(sigma), _ptr(snr), _ptr(t), _ptr(W),
                                              _stream()))
        return snr, t, W

    # ----------------------------------------------------------------- backward
    def backward(self, grad_y: torch.Tensor, x: torch.Tensor, need_x: bool = True,
                 need_w: bool = True, weights: Optional[torch.Tensor] = None):
        """(grad_x fp32 or None, grad_w fp64 or None) for the adjoint of dedisperse."""
        _dev_check(grad_y, "grad_y")
        _dev_check(x, "x")
        xb = x if x.dim() == 3 else x.unsqueeze(0)
        gb = grad_y if grad_y.dim() == 3 else grad_y.unsqueeze(0)
        gb = gb.contiguous().to(torch.float32)
        B, C, T = xb.shape
        nout = gb.shape[2]
        gx = torch.empty((B, C, T), dtype=torch.float32, device=x.device) if need_x else None
        gw = None
        if need_w and self.wmode != "unit":
            gw = torch.empty((C, self.ktaps) if self.wmode == "tap" else (C,), dtype=torch.float64,
                             device=x.device)
        wptr = None
        if weights is not None:
            weights = weights.contiguous().to(torch.float32)
            wptr = _ptr(weights)
        L.check(L.lib().dedisp_dedisperse_backward(
            self._h, _ptr(gb), nout, gb.stride(1), gb.stride(0), B, _ptr(xb), _TORCH_DT[x.dtype], T,
            xb.stride(1), xb.stride(0), _ptr(gx) if gx is not None else None,
            _ptr(gw) if gw is not None else None, wptr, _stream()))
        if gx is not None and x.dim() == 2:
            gx = gx[0]
        return gx, gw

    def gather(self, x: torch.Tensor, b, d, t, weights: Optional[torch.Tensor] = None):
        """Selected outputs y[b_e, d_e, t_e] (fp32) without computing the rest."""
        xb = x if x.dim() == 3 else x.unsqueeze(0)
        B, C, T = xb.shape
        bi, di, ti = [torch.as_tensor(v, dtype=torch.int32, device=x.device).contiguous() for v in (b, d, t)]
        out = torch.empty(bi.numel(), dtype=torch.float32, device=x.device)
        wptr = None
        if weights is not None:
            weights = weights.contiguous().to(torch.float32)
            wptr = _ptr(weights)
        L.check(L.lib().dedisp_dedisperse_gather(
            self._h, bi.numel(), _ptr(bi), _ptr(di), _ptr(ti), _ptr(xb), _TORCH_DT[x.dtype], T,
            xb.stride(1), xb.stride(0), B, _ptr(out), wptr, _stream()))
        return out

    def backward_sparse(self, x: torch.Tensor, b, d, t, val: torch.Tensor):
        """grad_w (fp64) for an output gradient that is non-zero only at (b_e, d_e, t_e)."""
        xb = x if x.dim() == 3 else x.unsqueeze(0)
        B, C, T = xb.shape
        bi, di, ti = [torch.as_tensor(v, dtype=torch.int32, device=x.device).contiguous() for v in (b, d, t)]
        v = val.contiguous().to(torch.float32)
        gw = torch.empty((C, self.ktaps) if self.wmode == "tap" else (C,), dtype=torch.float64,
                         device=x.device)
        L.check(L.lib().dedisp_backward_sparse(
            self._h, bi.numel(), _ptr(bi), _ptr(di), _ptr(ti), _ptr(v), _ptr(xb), _TORCH_DT[x.dtype],
            T, xb.stride(1), xb.stride(0), B, _ptr(gw), _stream()))
        return gw

    def set_tile(self, tile: int) -> None:
        L.check(L.lib().dedisp_set_tile(self._h, tile))

    def last_search_tile(self) -> int:
        """Tile configuration of the fused kernel used by the last search (-1: unfused)."""
        v = ctypes.c_int32()
        L.check(L.lib().dedisp_last_search_tile(self._h, ctypes.byref(v)))
        return v.value

    def fused_search(self) -> bool:
        return self.last_search_tile() >= 0

    def set_kernel_events(self, starts, stops) -> None:
        """Record torch.cuda.Event pairs around the dominant kernel of each search call
        (cycling over the pairs).  Events must already have been recorded once so that
        their HIP handles exist.  Pass empty lists to disable."""
        n = len(starts)
        a = (ctypes.c_void_p * max(n, 1))(*[e.cuda_event for e in starts])
        b = (ctypes.c_void_p * max(n, 1))(*[e.cuda_event for e in stops])
        self._events = (starts, stops, a, b)
        L.check(L.lib().dedisp_set_kernel_events(self._h, a, b, n))


def trial_dms(dm0: float, dm_max: float, eps: float, freq_ghz, chan_bw_ghz: float, dt_s: float,
              tau_av_s: float = 0.0, include_dm_tau: bool = False, k_dm: float = 0.0,
              cap: int = 100000) -> np.ndarray:
    """eq. trial DMs (Section 5.3), evaluated by the library."""
    f = np.ascontiguousarray(freq_ghz, dtype=np.float64)
    out = np.empty(cap, dtype=np.float64)
    n = ctypes.c_int32()
    L.check(L.lib().dedisp_trial_dms(dm0, dm_max, eps, len(f), _ptr(f), chan_bw_ghz, dt_s, tau_av_s,
                                     int(include_dm_tau), k_dm, cap, _ptr(out), ctypes.byref(n)))
    return out[:n.value].copy()


def _autotune(self, x: torch.Tensor, widths: Sequence[int], mean, sigma,
              work: Optional[torch.Tensor] = None) -> int:
    """Time every tile shape of the fused search on block x and keep the fastest
    for this plan (cached in the file named by DEDISP_TUNE_CACHE, if set)."""
    _dev_check(x, "x")
    C, T = x.shape
    w = self._widths(widths)
    m, s = (mean, sigma) if isinstance(mean, torch.Tensor) else self._meansig(mean, sigma, x.device)
    need = self.work_bytes(T, len(w))
    if work is None or work.numel() < need:
        work = torch.empty(need, dtype=torch.uint8, device=x.device)
    chosen = ctypes.c_int32()
    L.check(L.lib().dedisp_autotune(self._h, _ptr(x), T, x.stride(0), _ptr(w), len(w), _ptr(m),
                                    _ptr(s), _ptr(work), work.numel(), _stream(),
                                    ctypes.byref(chosen)))
    return chosen.value


Plan.autotune = _autotune


class Batch:
    """Many beams (each with its own plan and block length) searched by one
    launch over every beam's tiles; `run(..., graph=True)` replays a captured HIP graph."""

    def __init__(self, plans: Sequence[Plan], nsamp: Sequence[int], widths: Sequence[int]):
        self.plans = list(plans)
        n = np.ascontiguousarray(nsamp, dtype=np.int64)
        ps = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        w = np.ascontiguousarray(widths, dtype=np.int32)
        h = ctypes.c_void_p()
        L.check(L.lib().dedisp_batch_create(ctypes.byref(h), len(self.plans), ps, _ptr(n), _ptr(w),
                                            len(w)))
        self._h = h
        self.widths = w
        v = ctypes.c_size_t()
        L.check(L.lib().dedisp_batch_work_bytes(h, ctypes.byref(v)))
        self.work_bytes = v.value
        a, b = ctypes.c_int64(), ctypes.c_int64()
        L.check(L.lib().dedisp_batch_info(h, ctypes.byref(a), ctypes.byref(b)))
        self.total_trials, self.total_sums = a.value, b.value

    def close(self) -> None:
        if getattr(self, "_h", None):
            L.lib().dedisp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, xs: Sequence[torch.Tensor], mean: torch.Tensor, sigma: torch.Tensor,
            work: Optional[torch.Tensor] = None, outputs=None, graph: bool = False):
        """Best (snr, t, W) of every trial of every beam, concatenated in beam order."""
        for x in xs:
            _dev_check(x, "x")
        dev = xs[0].device
        ptrs = (ctypes.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        strides = np.ascontiguousarray([x.stride(0) for x in xs], dtype=np.int64)
        if work is None or work.numel() < self.work_bytes:
            work = torch.empty(self.work_bytes, dtype=torch.uint8, device=dev)
        if outputs is None:
            n = self.total_trials
            outputs = (torch.empty(n, dtype=torch.float64, device=dev),
                       torch.empty(n, dtype=torch.int32, device=dev),
                       torch.empty(n, dtype=torch.int32, device=dev))
        snr, t, W = outputs
        self._keep = (xs, mean, sigma, work, outputs, ptrs, strides)
        L.check(L.lib().dedisp_batch_run(self._h, ptrs, _ptr(strides), _ptr(mean), _ptr(sigma),
                                         _ptr(snr), _ptr(t), _ptr(W), _ptr(work), work.numel(),
                                         int(graph), _stream()))
        return snr, t, W
