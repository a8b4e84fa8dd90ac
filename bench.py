#!/usr/bin/env python3
"""Benchmark of the reverse-mode operator kernels on one MI355X.

Workload (one "step" = one pass over all of it, inputs resident in HBM):
  * reduce_by_index primal + VJP on n = 2^26 FP32 values ~ N(0,1), for the
    operators + and max (argmax ties to the lowest index), with m in
    {2^10, 2^16, 2^20} bins and bin indices uniform or Zipf(1.1): 12
    primal/VJP pairs;
  * scatter primal (save + scatter) and its adjoint (gather + zero +
    restore) with 2^24 unique int32 targets into a 2^26 FP32 array.

value = elements differentiated per second: each primal+VJP pair counts its
n elements (2^26 per histogram, 2^24 updates for the scatter), divided by
the step time.  The JSON line also carries the per-instance grad/primal
ratios ((primal + VJP) / primal), the roofline of the dominant kernel (timed
with HIP events on the stream it runs on) and the CPU oracle timed on a
bounded sample of the same inputs.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "VJP elems/s and % HBM peak; grad/primal time ratio; served p50/p99 latency"
HBM_PEAK_GBPS = 8000.0

N_HIST = 1 << 26
BINS = [1 << 10, 1 << 16, 1 << 20]
DISTS = ["uniform", "zipf"]
HIST_OPS = ["add", "max"]
N_SCAT, M_SCAT = 1 << 26, 1 << 24


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 21, help="elements per instance for the CPU oracle")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Algorithmic bytes moved per call (inputs read + outputs written once).
def hist_bytes(op, n, m):
    # primal: inds + vs; outputs hs (+ winner for max)
    return 8 * n + (8 if op == "max" else 4) * m


def hist_vjp_bytes(op, n, m):
    # add: inds read + vs_bar written (hs_bar is cache resident);
    # max: zero fill of vs_bar + winner/hs_bar reads and m scattered writes
    return 8 * n + 4 * m if op == "add" else 4 * n + 12 * m


def scatter_bytes(m):
    return 20 * m  # is, vs, xs[is] read; xs_saved, xs[is] written


def scatter_vjp_bytes(m):
    return 24 * m  # is, ys_bar[is], xs_saved read; vs_bar, ys_bar[is], ys[is] written


def traffic_for(kernel_key):
    """HBM bytes per launch from committed rocprofv3 counters, if they were
    taken on the current source of the kernel's file."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel_key)
    except Exception:
        return None
    if not rec:
        return None
    src = os.path.join(ROOT, rec["source"])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] if os.path.exists(src) else None
    return rec["bytes_per_launch"] if sha == rec.get("source_sha") else None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              "(multi-GPU sharding is design-only)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2202_10297_amd import capi, workloads

    capi.lib()
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    L = capi.lib()

    t0 = time.time()
    g = workloads.rng(0)
    vs_np = g.standard_normal(N_HIST, dtype=np.float32)
    vs = torch.from_numpy(vs_np).to(dev)
    inst = []
    for m in BINS:
        hb = torch.from_numpy(workloads.rng(m).standard_normal(m).astype(np.float32)).to(dev)
        for dist in DISTS:
            seed = 1000 + m.bit_length() * 10 + (dist == "zipf")
            gi = workloads.rng(seed)
            if dist == "uniform":
                ind_np = gi.integers(0, m, N_HIST, dtype=np.int32)
            else:
                ind_np = workloads.zipf_indices(N_HIST, m, 1.1, gi)
            inds = torch.from_numpy(ind_np).to(dev)
            for op in HIST_OPS:
                inst.append(dict(op=op, m=m, dist=dist, inds=inds, ind_np=ind_np if op == "add" else None, hb=hb))
            log(f"inputs m={m} {dist} ready ({time.time() - t0:.1f}s)")
    xs_np, is_np, sv_np, yb_np = workloads.scatter(N_SCAT, M_SCAT, "f32", seed=7)
    xs, is_, sv, ysb = (torch.from_numpy(a).to(dev) for a in (xs_np, is_np, sv_np, yb_np))
    log(f"inputs ready ({time.time() - t0:.1f}s)")

    # Preallocated outputs and workspaces: the timed loop only launches.
    stream = torch.cuda.current_stream(dev)
    sp = stream.cuda_stream
    OPC = {"add": capi.ADD, "max": capi.MAX}
    for it in inst:
        o, m = OPC[it["op"]], it["m"]
        it["hs"] = torch.empty(m, dtype=torch.float32, device=dev)
        it["winner"] = torch.empty(m, dtype=torch.int32, device=dev) if it["op"] == "max" else None
        nb = L.pvjp_hist_ws_bytes(o, capi.F32, N_HIST, m)
        it["ws"] = torch.zeros(nb, dtype=torch.uint8, device=dev)
        it["vsb"] = torch.empty(N_HIST, dtype=torch.float32, device=dev)
    saved = torch.empty(M_SCAT, dtype=torch.float32, device=dev)
    vsb_s = torch.empty(M_SCAT, dtype=torch.float32, device=dev)

    def p(t):
        return None if t is None else t.data_ptr()

    calls = []  # (key, fn, bytes, elems, kind)
    for it in inst:
        o, m = OPC[it["op"]], it["m"]
        key = f"hist_{it['op']}_m{m}_{it['dist']}"

        def prim(it=it, o=o, m=m):
            capi.call("pvjp_hist", o, capi.F32, p(it["inds"]), p(vs), N_HIST, m, p(it["hs"]), p(it["winner"]),
                      None, None, None, p(it["ws"]), it["ws"].numel(), sp)

        def vjp(it=it, o=o, m=m):
            capi.call("pvjp_hist_vjp", o, capi.F32, p(it["inds"]), None, N_HIST, m, p(it["winner"]), None, None,
                      p(it["hb"]), p(it["vsb"]), 0, sp)

        calls.append((key, "primal", prim, hist_bytes(it["op"], N_HIST, m), N_HIST))
        calls.append((key, "vjp", vjp, hist_vjp_bytes(it["op"], N_HIST, m), 0))

    def sprim():
        capi.call("pvjp_scatter", capi.F32, p(xs), N_SCAT, p(is_), p(sv), M_SCAT, p(saved), sp)

    def svjp():
        capi.call("pvjp_scatter_vjp", capi.F32, p(ysb), N_SCAT, p(is_), M_SCAT, p(vsb_s), 0, p(xs), p(saved), sp)

    calls.append(("scatter_m2^24_n2^26", "primal", sprim, scatter_bytes(M_SCAT), M_SCAT))
    calls.append(("scatter_m2^24_n2^26", "vjp", svjp, scatter_vjp_bytes(M_SCAT), 0))
    elems_per_step = sum(c[4] for c in calls)

    def step(evs=None):
        for i, (_, _, fn, _, _) in enumerate(calls):
            if evs is not None:
                evs[i][0].record(stream)
            fn()
            if evs is not None:
                evs[i][1].record(stream)

    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # Parity spot check on this run's output: the + adjoint is a gather.
    it0 = inst[0]
    idx = np.random.default_rng(1).integers(0, N_HIST, 4096)
    got = it0["vsb"].cpu().numpy()[idx]
    exp = it0["hb"].cpu().numpy()[it0["ind_np"][idx]]
    if not np.array_equal(got, exp):
        log("PARITY FAILURE in the + histogram adjoint")
        sys.exit(3)

    log(f"timing {args.steps} steps")
    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in calls]
           for _ in range(args.steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record(stream)
    for k in range(args.steps):
        step(evs[k])
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = start.elapsed_time(stop)
    ms_per_step = total_ms / args.steps

    per_call = np.array([[evs[k][i][0].elapsed_time(evs[k][i][1]) for i in range(len(calls))]
                         for k in range(args.steps)])
    avg = per_call.mean(0)
    detail = {}
    for i, (key, kind, _, nbytes, _) in enumerate(calls):
        d = detail.setdefault(key, {})
        d[f"{kind}_ms"] = round(float(avg[i]), 4)
        d[f"{kind}_GBps"] = round(nbytes / (avg[i] * 1e-3) / 1e9, 1)
    for d in detail.values():
        d["grad_over_primal"] = round((d["primal_ms"] + d["vjp_ms"]) / d["primal_ms"], 3)

    dom = int(np.argmax(avg))
    dkey, dkind, _, dbytes, _ = calls[dom]
    achieved = dbytes / (avg[dom] * 1e-3) / 1e9
    kernel_name = {"primal": "hist_acc_kernel" if dkey.startswith("hist") else "scatter_kernel",
                   "vjp": "hist_vjp" if dkey.startswith("hist") else "scatter_vjp_kernel"}[dkind]
    roof = {
        "bound": "hbm",
        "kernel": f"{dkey}:{dkind} ({kernel_name})",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBPS, 4),
        "traffic": traffic_for(f"{dkey}:{dkind}"),
        "alg_bytes_per_launch": dbytes,
        "avg_launch_ms": round(float(avg[dom]), 4),
    }

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_sample, vs_np, inst, xs_np, is_np, sv_np, yb_np)

    out = {
        "metric": METRIC,
        "value": round(elems_per_step / (ms_per_step * 1e-3), 1),
        "unit": "elems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "reduce_by_index (+, max) primal+VJP n=2^26 FP32, m in {2^10,2^16,2^20}, "
                        "uniform and Zipf(1.1) indices; scatter primal+VJP 2^24 unique targets into 2^26 FP32",
            "elems_per_step": elems_per_step,
            "parallelism": "single GPU",
        },
        "wall_s_timed": round(wall, 3),
        "grad_over_primal_max": max(d["grad_over_primal"] for d in detail.values()),
        "served_latency": None,
        "roofline": roof,
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(ns, vs_np, inst, xs_np, is_np, sv_np, yb_np):
    """The oracle (single-threaded, FP64 tape) on the first `ns` elements of
    every histogram instance and on the scatter restricted to targets below
    `ns` (primal + VJP each), scaled to elements per second."""
    sys.path.insert(0, ROOT)
    import oracle

    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    vsn = vs_np[:ns]
    elems = 0
    t0 = time.perf_counter()
    for it in inst:
        ind = it["inds"][:ns].cpu().numpy()
        hb = it["hb"].cpu().numpy()
        oracle.hist(it["op"], ind, vsn, it["m"])
        oracle.hist_vjp(it["op"], ind, vsn, hb)
        elems += ns
    sel = is_np[is_np < ns][: ns // 4]
    oracle.scatter(xs_np[:ns], sel, sv_np[: sel.size])
    oracle.scatter_vjp(sel, yb_np[:ns])
    elems += sel.size
    dt = time.perf_counter() - t0
    return {
        "value": round(elems / dt, 1),
        "unit": "elems/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first {ns} elements of each of the 12 histogram instances (+ and max, primal and taped VJP) "
                  f"and a scatter of {sel.size} targets into {ns}; {dt:.1f}s",
    }


if __name__ == "__main__":
    main()
