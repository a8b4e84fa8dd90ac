"""Serving loop for gradient requests of mixed kinds and sizes.

Requests are VJP evaluations against primal inputs that stay resident on the
device (registered once in a ``Pool``); a request carries only its kind, the
handle of its resident instance and the handle of its output adjoint.  Kinds:

* ``scan``: the reverse sweep of a linear-recurrence scan (its checkpoint is
  resident too), ``pvjp_linrec_scan_vjp``;
* ``hist``: the adjoint of a + histogram, ``pvjp_hist_vjp``;
* ``gmm``: the full gradient of a Gaussian-mixture log-likelihood (its
  per-point LSE checkpoint is resident), ``pvjp_gmm_vjp``.

Scheduling (continuous admission, not a queue alone): requests arriving while
others run wait in a FIFO; whenever a slot (a HIP stream with its own
workspaces) is free and the request's HBM footprint (its outputs and
workspace) fits the budget beside the requests in flight, it is admitted:
its outputs are allocated on its slot's stream and its kernels are launched
there, overlapping on the device with the other slots.  Completion is observed
by polling an event recorded after the request's kernels; latency is
completion minus arrival.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import capi, ops, workloads
from .ops import _ptr

KINDS = ("scan", "hist", "gmm")
GMM_D, GMM_K = 32, 50


# ----------------------------------------------------------------- the pool
@dataclass
class Instance:
    kind: str
    n: int
    m: int = 0
    tensors: dict = field(default_factory=dict)


class Pool:
    """Resident primal inputs (and checkpoints) for each request kind."""

    def __init__(self, per_kind=16, seed=0, device="cuda", scan_range=(10 ** 3, 10 ** 7),
                 hist_range=(10 ** 4, 10 ** 7), hist_bins=(12, 18), gmm_range=(10 ** 3, 10 ** 5), ybar_variants=2,
                 device_gen=False):
        self.device = torch.device(device)
        self.inst = {k: [] for k in KINDS}
        g = workloads.rng(seed)
        logu = lambda lo, hi: int(np.exp(g.uniform(np.log(lo), np.log(hi))))
        t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(self.device)
        if device_gen:
            self._device_pool(per_kind, seed, logu, g, scan_range, hist_range, hist_bins, gmm_range, ybar_variants)
            return
        for i in range(per_kind):
            n = logu(*scan_range)
            a, b, _, _ = workloads.linrec(n, "f32", seed=seed * 1000 + i)
            da, db = t(a), t(b)
            _, _, ck = ops.linrec_scan(da, db)
            yb = []
            for v in range(ybar_variants):
                _, _, ya_, yb_ = workloads.linrec(n, "f32", seed=seed * 1000 + i + 7919 * (v + 1))
                yb.append((t(ya_), t(yb_)))
            self.inst["scan"].append(Instance("scan", n, tensors=dict(a=da, b=db, ckpt=ck, ybar=yb)))
        for i in range(per_kind):
            n = logu(*hist_range)
            m = 1 << int(g.integers(hist_bins[0], hist_bins[1] + 1))
            inds, _, _ = workloads.hist(n, m, "zipf", "f32", seed=seed * 2000 + i)
            yb = [t(workloads.rng(seed * 2000 + i + 31 * (v + 1)).standard_normal(m).astype(np.float32))
                  for v in range(ybar_variants)]
            self.inst["hist"].append(Instance("hist", n, m, tensors=dict(inds=t(inds), ybar=yb)))
        for i in range(per_kind):
            N = logu(*gmm_range)
            X, al, mu, q, l = workloads.gmm(N, GMM_D, GMM_K, seed=seed * 3000 + i)
            P = [t(x) for x in (X, al, mu, q, l)]
            _, lse = ops.gmm_objective(*P)
            yb = [1.0 + 0.5 * v for v in range(ybar_variants)]
            self.inst["gmm"].append(Instance("gmm", N, tensors=dict(X=P[0], alpha=P[1], mu=P[2], q=P[3], l=P[4],
                                                                     lse=lse, ybar=yb)))
        torch.cuda.synchronize(self.device)

    def _device_pool(self, per_kind, seed, logu, g, scan_range, hist_range, hist_bins, gmm_range, ybar_variants):
        """The same instance sizes and input distributions as the host-drawn
        pool, drawn on the device with torch's generator (a large pool's
        Zipf indices would take minutes on the host)."""
        dev = self.device
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed + 77)
        f32 = torch.float32
        randn = lambda *sh: torch.randn(*sh, dtype=f32, device=dev, generator=gen)
        for _ in range(per_kind):
            n = logu(*scan_range)
            a = torch.rand(n, dtype=f32, device=dev, generator=gen) * 0.5 + 0.5
            b = randn(n)
            _, _, ck = ops.linrec_scan(a, b)
            yb = [(randn(n), randn(n)) for _ in range(ybar_variants)]
            self.inst["scan"].append(Instance("scan", n, tensors=dict(a=a, b=b, ckpt=ck, ybar=yb)))
        for _ in range(per_kind):
            n = logu(*hist_range)
            m = 1 << int(g.integers(hist_bins[0], hist_bins[1] + 1))
            k = torch.arange(1, m + 1, dtype=torch.float64, device=dev)
            cdf = torch.cumsum(k ** -1.1, 0)
            cdf /= cdf[-1].clone()
            u = torch.rand(n, dtype=torch.float64, device=dev, generator=gen)
            r = torch.searchsorted(cdf, u, right=True).clamp_(max=m - 1)
            perm = torch.randperm(m, device=dev, generator=gen)
            inds = perm[r].to(torch.int32)
            yb = [randn(m) for _ in range(ybar_variants)]
            self.inst["hist"].append(Instance("hist", n, m, tensors=dict(inds=inds, ybar=yb)))
        tri = GMM_D * (GMM_D - 1) // 2
        for _ in range(per_kind):
            N = logu(*gmm_range)
            X, al, mu = randn(N, GMM_D), randn(GMM_K), randn(GMM_K, GMM_D)
            q, l = randn(GMM_K, GMM_D) * 0.1, randn(GMM_K, tri) * 0.1
            _, lse = ops.gmm_objective(X, al, mu, q, l)
            yb = [1.0 + 0.5 * v for v in range(ybar_variants)]
            self.inst["gmm"].append(Instance("gmm", N, tensors=dict(X=X, alpha=al, mu=mu, q=q, l=l, lse=lse,
                                                                     ybar=yb)))
        torch.cuda.synchronize(dev)

    def max_n(self, kind):
        return max(i.n for i in self.inst[kind])


# ---------------------------------------------------------------- requests
@dataclass
class Request:
    rid: int
    arrival: float  # seconds from the start of the trace
    kind: str
    inst: int
    ybar: int
    admitted: float = -1.0
    done: float = -1.0
    outputs: tuple = ()
    event: object = None
    slot: int = -1
    footprint: int = 0


def make_burst(pool: Pool, count: int, seed=0, mix=(1 / 3, 1 / 3, 1 / 3)):
    """`count` requests that all arrive at time 0 (a saturating load)."""
    g = workloads.rng(seed + 54321)
    kinds = g.choice(len(KINDS), size=count, p=np.asarray(mix) / np.sum(mix))
    reqs = []
    for i, k in enumerate(kinds):
        kind = KINDS[int(k)]
        reqs.append(Request(i, 0.0, kind, int(g.integers(0, len(pool.inst[kind]))), int(g.integers(0, 2))))
    return reqs


def make_trace(pool: Pool, rate=2000.0, duration=30.0, seed=0, mix=(1 / 3, 1 / 3, 1 / 3)):
    """Poisson arrivals at `rate` per second for `duration` seconds."""
    g = workloads.rng(seed + 12345)
    n = int(rate * duration * 1.2) + 16
    t = np.cumsum(g.exponential(1.0 / rate, n))
    t = t[t < duration]
    kinds = g.choice(len(KINDS), size=t.size, p=np.asarray(mix) / np.sum(mix))
    reqs = []
    for i, (ti, k) in enumerate(zip(t, kinds)):
        kind = KINDS[int(k)]
        inst = int(g.integers(0, len(pool.inst[kind])))
        reqs.append(Request(i, float(ti), kind, inst, int(g.integers(0, 2))))
    return reqs


# ------------------------------------------------------------------ server
class Server:
    def __init__(self, pool: Pool, slots=8, budget_bytes=64 << 30, keep_outputs=False):
        self.pool = pool
        self.dev = pool.device
        self.nslots = int(slots)
        self.budget = int(budget_bytes)
        self.keep = keep_outputs
        # Default-priority streams only.
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(self.nslots)]
        L = capi.lib()
        # Workspace sizes are not monotone in the problem size: take the
        # maximum over the resident instances.
        self.ws_scan_bytes = max(L.pvjp_linrec_scan_vjp_ws_bytes(capi.F32, i.n) for i in pool.inst["scan"])
        self.ws_gmm_bytes = max(L.pvjp_gmm_ws_bytes(i.n, GMM_D, GMM_K) for i in pool.inst["gmm"])
        self.ws = []
        for _ in range(self.nslots):
            self.ws.append(dict(scan=self._zeros(self.ws_scan_bytes), gmm=self._zeros(self.ws_gmm_bytes)))

    def _zeros(self, nbytes):
        buf = torch.zeros(nbytes + 256, dtype=torch.uint8, device=self.dev)
        off = (-buf.data_ptr()) % 256
        return buf[off:off + nbytes]

    # footprint of a request: outputs (+ the share of workspace it occupies)
    def footprint(self, r: Request) -> int:
        it = self.pool.inst[r.kind][r.inst]
        if r.kind == "scan":
            return 2 * 4 * it.n + self.ws_scan_bytes
        if r.kind == "hist":
            return 4 * it.n
        tri = GMM_D * (GMM_D - 1) // 2
        return 4 * GMM_K * (1 + 2 * GMM_D + tri) + self.ws_gmm_bytes

    def _launch(self, r: Request, slot: int):
        it = self.pool.inst[r.kind][r.inst]
        T = it.tensors
        st = self.streams[slot]
        sp = st.cuda_stream
        with torch.cuda.stream(st):
            if r.kind == "scan":
                ya, yb = T["ybar"][r.ybar]
                ab = torch.empty(it.n, dtype=torch.float32, device=self.dev)
                bb = torch.empty(it.n, dtype=torch.float32, device=self.dev)
                ws = self.ws[slot]["scan"]
                capi.call("pvjp_linrec_scan_vjp", capi.F32, _ptr(T["a"]), _ptr(T["b"]), _ptr(ya), _ptr(yb), it.n,
                          _ptr(T["ckpt"]), _ptr(ab), _ptr(bb), 0, _ptr(ws), ws.numel(), sp)
                r.outputs = (ab, bb)
            elif r.kind == "hist":
                vb = torch.empty(it.n, dtype=torch.float32, device=self.dev)
                capi.call("pvjp_hist_vjp", capi.ADD, capi.F32, _ptr(T["inds"]), None, it.n, it.m, None, None, None,
                          _ptr(T["ybar"][r.ybar]), _ptr(vb), 0, sp)
                r.outputs = (vb,)
            else:
                outs = tuple(torch.empty_like(T[k]) for k in ("alpha", "mu", "q", "l"))
                ws = self.ws[slot]["gmm"]
                capi.call("pvjp_gmm_vjp", _ptr(T["X"]), it.n, GMM_D, GMM_K, _ptr(T["alpha"]), _ptr(T["mu"]),
                          _ptr(T["q"]), _ptr(T["l"]), float(T["ybar"][r.ybar]), _ptr(T["lse"]), None,
                          *[_ptr(o) for o in outs], 0, _ptr(ws), ws.numel(), sp)
                r.outputs = outs
            ev = torch.cuda.Event()
            ev.record(st)
            r.event = ev

    def run(self, trace, warmup=0.0, idle_sleep=20e-6):
        """Replays `trace` in real time; returns statistics over requests
        arriving at or after `warmup` seconds."""
        pending = list(trace)
        pending.sort(key=lambda r: r.arrival)
        queue = []
        inflight = [None] * self.nslots
        used = 0
        done = []
        max_inflight = 0
        admit_waits = 0
        head = 0
        torch.cuda.synchronize(self.dev)
        t0 = time.perf_counter()
        while head < len(pending) or queue or any(x is not None for x in inflight):
            now = time.perf_counter() - t0
            while head < len(pending) and pending[head].arrival <= now:
                queue.append(pending[head])
                head += 1
            # completions
            for s, r in enumerate(inflight):
                if r is not None and r.event.query():
                    r.done = time.perf_counter() - t0
                    used -= r.footprint
                    if not self.keep:
                        r.outputs = ()
                    r.event = None
                    inflight[s] = None
                    done.append(r)
            # admissions (FIFO by arrival)
            while queue:
                free = [s for s in range(self.nslots) if inflight[s] is None]
                if not free:
                    break
                r = queue[0]
                fp = self.footprint(r)
                if used + fp > self.budget:
                    if used == 0 and fp > self.budget:
                        raise RuntimeError(f"request {r.rid} needs {fp} bytes, above the budget")
                    admit_waits += 1
                    break
                queue.pop(0)
                r.footprint = fp
                used += fp
                r.slot = free[0]
                r.admitted = time.perf_counter() - t0
                self._launch(r, free[0])
                inflight[free[0]] = r
            max_inflight = max(max_inflight, sum(x is not None for x in inflight))
            if head < len(pending) and not queue and all(x is None for x in inflight):
                time.sleep(max(0.0, min(pending[head].arrival - (time.perf_counter() - t0), 1e-3)))
            elif idle_sleep:
                time.sleep(idle_sleep)
        wall = time.perf_counter() - t0
        meas = [r for r in done if r.arrival >= warmup]
        lat = np.array([r.done - r.arrival for r in meas]) * 1e3
        span = (max(r.done for r in meas) - min(r.arrival for r in meas)) if meas else 0.0
        elems = sum(self.pool.inst[r.kind][r.inst].n for r in meas)
        stats = {
            "requests": len(meas),
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_ms": float(lat.mean()) if len(lat) else None,
            "throughput_rps": len(meas) / span if span > 0 else None,
            "elems_per_s": elems / span if span > 0 else None,
            "max_inflight": max_inflight,
            "admission_waits": admit_waits,
            "slots": self.nslots,
            "budget_bytes": self.budget,
            "wall_s": wall,
        }
        by_kind = {}
        for k in KINDS:
            lk = np.array([r.done - r.arrival for r in meas if r.kind == k]) * 1e3
            if lk.size:
                by_kind[k] = {"n": int(lk.size), "p50_ms": float(np.percentile(lk, 50)),
                              "p99_ms": float(np.percentile(lk, 99))}
        stats["by_kind"] = by_kind
        return stats, done
