"""Segmented batches: many scan VJPs and sum-reduce VJPs of uneven lengths in
one persistent launch, with autotuned tile size and grid, captured in a HIP
graph and replayed.

A ``SegPlan`` fixes the segment table (uploaded once into its workspace by
``pvjp_seg_prepare``).  ``SegPlan.scan`` runs the segmented primal (and
writes the checkpoint the return sweep recomputes from); ``SegPlan.vjp`` runs
``pvjp_seg_batch_vjp``; ``SegPlan.capture`` records that call into a graph
whose ``replay`` re-launches it without host overhead.  The library's
lookback state resets itself at the end of every launch, so replays need no
memset nodes.
"""
from __future__ import annotations

import numpy as np
import torch

from . import capi
from .ops import _after_lookback, _check_values, _dt, _ptr, _stream

TILES = (1024, 2048, 4096)
DEFAULT_TILE = 4096


def default_grid(device=None) -> int:
    """Persistent grid: a few workgroups per compute unit."""
    props = torch.cuda.get_device_properties(device)
    return 4 * props.multi_processor_count


class SegPlan:
    def __init__(self, lengths, dtype=torch.float32, device="cuda", tile=None, grid=None, tune=False,
                 tune_inputs=None):
        lengths = np.asarray(lengths, dtype=np.int64)
        if lengths.ndim != 1 or lengths.size == 0 or np.any(lengths < 1):
            raise ValueError("segment lengths must be a non-empty list of positive integers")
        self.lengths = lengths
        self.offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
        self.nseg = int(lengths.size)
        self.total = int(self.offsets[-1])
        self.dtype = dtype
        self.device = torch.device(device)
        if tune and (tile is None or grid is None):
            from . import tune as _tune

            tile, grid = _tune.seg_config(self, tune_inputs)
        self.tile = int(tile or DEFAULT_TILE)
        self.grid = int(grid or default_grid(self.device))
        self._prepare()
        self._graph = None

    # -------------------------------------------------------------- setup
    def _prepare(self):
        L = capi.lib()
        nb = L.pvjp_seg_ws_bytes(self.total, self.nseg, self.tile)
        if nb == 0:
            raise ValueError("invalid segment plan")
        buf = torch.zeros(nb + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        self.ws = buf[off:off + nb]
        offs = np.ascontiguousarray(self.offsets)
        capi.call("pvjp_seg_prepare", offs.ctypes.data, self.nseg, self.tile, _ptr(self.ws), nb,
                  _stream(self.device))

    def retile(self, tile: int, grid: int | None = None):
        if tile not in TILES:
            raise ValueError(f"tile must be one of {TILES}")
        self.tile = tile
        if grid is not None:
            self.grid = int(grid)
        self._prepare()
        self._graph = None

    def ckpt_len(self) -> int:
        return 2 * capi.lib().pvjp_linrec_ckpt_len(self.total)

    # -------------------------------------------------------------- calls
    def scan(self, a, b, outputs=True):
        """Segmented primal: returns (A, B, ckpt); A, B are None when
        outputs=False (checkpoint only)."""
        A = torch.empty_like(a) if outputs else None
        B = torch.empty_like(b) if outputs else None
        ck = torch.empty(self.ckpt_len(), dtype=a.dtype, device=a.device)
        _check_values(a, b)
        capi.call("pvjp_seg_linrec_scan", _dt(a), _ptr(a), _ptr(b), self.total, self.nseg, self.tile, _ptr(A),
                  _ptr(B), _ptr(ck), _ptr(self.ws), self.ws.numel(), _stream(a.device))
        _after_lookback(self.ws)
        return A, B, ck

    def vjp(self, a=None, b=None, yA_bar=None, yB_bar=None, ckpt=None, a_bar=None, b_bar=None, sum_ybar=None,
            sum_xbar=None, accumulate=False):
        """The persistent batched return sweep; outputs are written in place
        into a_bar, b_bar and sum_xbar (allocated if None)."""
        ref = a if a is not None else sum_ybar
        if a is not None:
            if a_bar is None:
                a_bar = (torch.zeros_like if accumulate else torch.empty_like)(a)
            if b_bar is None:
                b_bar = (torch.zeros_like if accumulate else torch.empty_like)(b)
        if sum_ybar is not None and sum_xbar is None:
            sum_xbar = (torch.zeros if accumulate else torch.empty)(self.total, dtype=sum_ybar.dtype,
                                                                   device=sum_ybar.device)
        capi.call("pvjp_seg_batch_vjp", _dt(ref), _ptr(a), _ptr(b), _ptr(yA_bar), _ptr(yB_bar), self.total,
                  self.nseg, self.tile, _ptr(ckpt), _ptr(a_bar), _ptr(b_bar), _ptr(sum_ybar), _ptr(sum_xbar),
                  int(accumulate), self.grid, _ptr(self.ws), self.ws.numel(), _stream(ref.device))
        _after_lookback(self.ws)
        return a_bar, b_bar, sum_xbar

    # -------------------------------------------------------------- graphs
    def capture(self, **kwargs):
        """Records one vjp(**kwargs) call (fixed buffers) into a HIP graph."""
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            self.vjp(**kwargs)  # warm-up outside the graph on the capture stream
        torch.cuda.current_stream(self.device).wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.vjp(**kwargs)
        self._graph = g
        return g

    def replay(self):
        if self._graph is None:
            raise RuntimeError("capture() first")
        self._graph.replay()
