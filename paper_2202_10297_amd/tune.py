"""Autotuner for the segmented batch launch: tile size (elements per tile,
i.e. items per thread at 256 threads) and persistent grid size.

Candidates are timed on the plan's own segment table with HIP events (a few
warm-up launches, then the median of several timed launches), and the winner
is cached in a JSON file keyed by device architecture, dtype and a coarse
signature of the segment-length distribution.  The cache lives at
$PVJP_TUNE_CACHE, else ~/.cache/pvjp/tune.json; if that cannot be written the
result is kept in memory only.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

TILES = (1024, 2048, 4096)
GRIDS_PER_CU = (1, 2, 4, 8)

_mem: dict = {}


def cache_path() -> str:
    return os.environ.get("PVJP_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "pvjp", "tune.json"))


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except Exception:
        return {}


def _store(d: dict):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def signature(plan) -> str:
    arch = torch.cuda.get_device_properties(plan.device).gcnArchName.split(":")[0]
    L = plan.lengths
    q = np.percentile(L, [10, 50, 90]) if L.size else [0, 0, 0]
    b = lambda x: int(np.log2(max(1.0, float(x))))  # power-of-two buckets
    dt = "f64" if plan.dtype == torch.float64 else "f32"
    return f"seg:{arch}:{dt}:n{b(plan.total)}:s{b(plan.nseg)}:q{b(q[0])}-{b(q[1])}-{b(q[2])}"


def _time(fn, warm=2, reps=5) -> float:
    for _ in range(warm):
        fn()
    ts = []
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        e.synchronize()
        ts.append(s.elapsed_time(e))
    return float(np.median(ts))


def seg_config(plan, inputs=None, force=False):
    """Returns (tile, grid) for the plan, tuning on first use.

    `inputs` is a dict of device tensors for SegPlan.vjp (a, b, yA_bar,
    yB_bar, ckpt, a_bar, b_bar, sum_ybar, sum_xbar); without it, zero-filled
    stand-ins of the right sizes are used (the kernels' cost does not depend on
    the values)."""
    key = signature(plan)
    cache = _load()
    cache.update(_mem)
    if key in cache and not force:
        return tuple(cache[key])
    from .batch import SegPlan

    dev = plan.device
    if inputs is None:
        z = lambda n: torch.zeros(n, dtype=plan.dtype, device=dev)
        inputs = dict(a=z(plan.total), b=z(plan.total), yA_bar=z(plan.total), yB_bar=z(plan.total),
                      a_bar=z(plan.total), b_bar=z(plan.total), sum_ybar=z(plan.nseg), sum_xbar=z(plan.total))
    ncu = torch.cuda.get_device_properties(dev).multi_processor_count
    best = None
    for tile in TILES:
        p = SegPlan(plan.lengths, plan.dtype, dev, tile=tile, grid=ncu)
        kw = dict(inputs)
        if kw.get("a") is not None:
            _, _, kw["ckpt"] = p.scan(kw["a"], kw["b"], outputs=False)
        for g in GRIDS_PER_CU:
            p.grid = g * ncu
            t = _time(lambda: p.vjp(**kw))
            if best is None or t < best[0]:
                best = (t, tile, g * ncu)
    result = (best[1], best[2])
    _mem[key] = result
    cache[key] = result
    _store(cache)
    return result
