"""Streams that arrive in blocks (the real-time setting of Section 2.1).

The dedispersion sum at an output needs the `max_span` samples from it on, and a
boxcar window of width W the W - 1 outputs after its start, so the only state a
stream carries from one block to the next is the tail of the samples already seen:
`max_span - 1` samples for the dedispersed series, `max_span - 1 + W_max - 1` for the
search.  Each block is processed together with that tail by the library's
dedispersion or fused search; the per-trial best over the blocks is kept on the device
by `dedisp_merge_candidates`.  Only the tail copy (device to device) happens here.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib as L
from .api import Plan, _dev_check, _ptr, _stream


class _Tail:
    """The last `keep` samples of the stream seen so far, and the stream index of the
    first of them."""

    def __init__(self, keep: int):
        self.keep = keep
        self.buf: Optional[torch.Tensor] = None
        self.start = 0

    def join(self, chunk: torch.Tensor) -> torch.Tensor:
        _dev_check(chunk, "chunk")
        if self.buf is None or self.buf.shape[1] == 0:
            return chunk
        return torch.cat([self.buf, chunk], dim=1)

    def advance(self, x: torch.Tensor) -> None:
        """x (the tail joined with the new block) becomes the seen stream's end."""
        n = x.shape[1]
        k = min(self.keep, n)
        self.start += n - k
        self.buf = x[:, n - k:].clone()


class StreamDedisperser:
    """Dedisperse a stream block by block: push() returns the dedispersed outputs the
    block completes (y[d, t] for stream outputs t0 .. t0 + y.shape[1] - 1) and t0, or
    (None, t0) while fewer than max_span samples have arrived.  The outputs of
    consecutive calls follow one another without gap or overlap, and equal the
    dedispersion of the whole stream."""

    def __init__(self, plan: Plan, out_dtype: Optional[torch.dtype] = None):
        self.plan = plan
        self.out_dtype = out_dtype
        self._tail = _Tail(plan.max_span - 1)

    def push(self, chunk: torch.Tensor):
        x = self._tail.join(chunk)
        t0 = self._tail.start
        if x.shape[1] < self.plan.max_span:
            self._tail.buf, self._tail.start = x.clone(), t0
            return None, t0
        y = self.plan.dedisperse(x, out_dtype=self.out_dtype)
        self._tail.advance(x)
        return y, t0


class StreamSearch:
    """Fused search of a stream block by block.  push() searches the block with the
    tail of the stream before it and returns that block's per-trial best (snr, t, W)
    and t0, the stream index of the block's first output (the block's starts t count
    from it), or None while fewer than max_span + W_max - 1 samples have arrived.
    best() is the per-trial best over everything pushed so far (snr f64, t i64, W i32
    device tensors; (-inf, -1, 0) for a trial with no window yet), which equals the
    search of the whole stream so far."""

    def __init__(self, plan: Plan, widths: Sequence[int], mean, sigma):
        self.plan = plan
        self.widths = [int(w) for w in widths]
        dev = mean.device if isinstance(mean, torch.Tensor) else torch.device("cuda")
        self.mean = torch.as_tensor(mean, dtype=torch.float64, device=dev).contiguous()
        self.sigma = torch.as_tensor(sigma, dtype=torch.float64, device=dev).contiguous()
        self.wmax = max(self.widths)
        self._tail = _Tail(plan.max_span - 1 + self.wmax - 1)
        self._snr = torch.full((plan.ndm,), float("-inf"), dtype=torch.float64, device=dev)
        self._t = torch.full((plan.ndm,), -1, dtype=torch.int64, device=dev)
        self._w = torch.zeros(plan.ndm, dtype=torch.int32, device=dev)
        self._work = None

    def push(self, chunk: torch.Tensor):
        x = self._tail.join(chunk)
        t0 = self._tail.start
        if x.shape[1] < self.plan.max_span + self.wmax - 1:
            self._tail.buf, self._tail.start = x.clone(), t0
            return None
        need = self.plan.work_bytes(x.shape[1], len(self.widths))
        if self._work is None or self._work.numel() < need:
            self._work = torch.empty(need, dtype=torch.uint8, device=x.device)
        snr, t, w = self.plan.search(x, self.widths, self.mean, self.sigma, work=self._work)
        L.check(L.lib().dedisp_merge_candidates(self.plan.ndm, _ptr(snr), _ptr(t), _ptr(w),
                                                ctypes.c_int64(t0), _ptr(self._snr),
                                                _ptr(self._t), _ptr(self._w), _stream()))
        self._tail.advance(x)
        return snr, t, w, t0

    def best(self):
        return self._snr, self._t, self._w
