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
COPY_N = 1 << 28


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 23, help="elements per instance for the CPU oracle")
    ap.add_argument("--skip", default="", help="comma list of extra workloads to skip: reduce_map,reduce_generic,scan_generic,jvp,kmeans,"
                         "gather_map,scan_batched,sparse_kmeans,hist_lae,hist_generic,scan,gmm,batch,serve")
    ap.add_argument("--only", default="",
                    help="run just this one extra workload (for profiling) and print its JSON instead of the "
                         "benchmark line")
    ap.add_argument("--serve-seconds", type=float, default=30.0, help="measured seconds of the serving trace")
    ap.add_argument("--ingest-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn the counter_collection.csv files of a FETCH_SIZE and a WRITE_SIZE run into "
                         "profiles/traffic.json (no GPU needed), then exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain streaming kernel over 2^28 FP32 (1 GiB read, 1 GiB written), whose "
                         "FETCH_SIZE/WRITE_SIZE counters scale the counters of the other kernels, then a gather of "
                         "2^21 whole 128-byte rows in random order (256 MiB read at random, 16 MiB of indices, "
                         "256 MiB written in order), whose counters calibrate random-order reads")
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


def call_order():
    """(instance key, primal|vjp) of the step's library calls, in launch order."""
    out = []
    for m in BINS:
        for dist in DISTS:
            for op in HIST_OPS:
                out += [(f"hist_{op}_m{m}_{dist}", "primal"), (f"hist_{op}_m{m}_{dist}", "vjp")]
    return out + [("scatter_m2^24_n2^26", "primal"), ("scatter_m2^24_n2^26", "vjp")]


# First kernel of each kind of library call: a new call starts at each one.
CALL_START_KERNELS = ("hist_acc_kernel", "hist_init_kernel", "hpart_tile_kernel", "hist_vjp_add_vec_kernel",
                      "hist_vjp_add_lds_kernel", "hist_vjp_add_kernel", "fill_zero_vec_kernel", "sp_count1_kernel",
                      "sp_clear_kernel")
MAIN_LINE_PREFIXES = ("hist_", "hpart_", "fill_zero", "sp_")
CALL_SOURCE = {"hist": "paper_2202_10297_amd/csrc/hist.hip", "scatter": "paper_2202_10297_amd/csrc/scatter_plan.hip"}
GATHER_ROWS = 1 << 21  # 128-byte rows of the random-order gather calibration (256 MiB)


def _short_kernel(name):
    base = name.split("(")[0].split("<")[0]
    return base.rsplit("::", 1)[-1].replace("void ", "").strip()


def _sha16(rel):
    return hashlib.sha256(open(os.path.join(ROOT, rel), "rb").read()).hexdigest()[:16]


def ingest_pmc(fetch_csv, write_csv):
    """HBM bytes per library call from one `--pmc FETCH_SIZE` and one
    `--pmc WRITE_SIZE` run of `bench.py --steps 1 --warmup 0
    --copy-calibration`.  Both counters are in KiB per dispatch; each is
    scaled by (bytes the calibration kernel moves) / (what the counter read
    for it), then summed over the kernels of each call.  Writes
    profiles/traffic.json."""
    import csv

    def per_dispatch(path):
        rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Dispatch_Id"]))
        return [(r["Kernel_Name"], float(r["Counter_Value"]) * 1024.0) for r in rows]

    out = {}
    scale = {}
    groups_by = {}
    for what, path in (("fetch", fetch_csv), ("write", write_csv)):
        d = per_dispatch(path)
        cal = [v for name, v in d if "neg_kernel" in name]
        if not cal:
            raise SystemExit(f"{path}: no calibration kernel (run bench.py with --copy-calibration)")
        scale[what] = (4.0 * COPY_N) / (sum(cal) / len(cal))
        gat = [v for name, v in d if "vectorized_gather_kernel" in name]
        if gat:  # random-order whole rows: reads 256 MiB + 8-byte indices, writes 256 MiB
            known = 128.0 * GATHER_ROWS + (8.0 * GATHER_ROWS if what == "fetch" else 0.0)
            scale["gather_" + what] = known / (sum(gat) / len(gat))
        groups = []
        for name, v in d:
            if "pvjp::" not in name:
                continue
            short = _short_kernel(name)
            if not short.startswith(MAIN_LINE_PREFIXES):
                break  # the other workloads run after the main line
            if short in CALL_START_KERNELS or not groups:
                groups.append([])
            groups[-1].append((short, v))
        groups_by[what] = groups
    order = call_order()
    for what in ("fetch", "write"):
        if len(groups_by[what]) != len(order):
            raise SystemExit(f"{what}: {len(groups_by[what])} calls found, expected {len(order)}")
    for i, (key, kind) in enumerate(order):
        src = CALL_SOURCE["scatter" if key.startswith("scatter") else "hist"]
        fb = sum(v for _, v in groups_by["fetch"][i]) * scale["fetch"]
        wb = sum(v for _, v in groups_by["write"][i]) * scale["write"]
        out[f"{key}:{kind}"] = {
            "source": src,
            "source_sha": _sha16(src),
            "kernels": [k for k, _ in groups_by["fetch"][i]],
            "fetch_bytes": round(fb),
            "write_bytes": round(wb),
            "bytes_per_launch": round(fb + wb),
        }
        if "gather_fetch" in scale:  # the same counters read with the random-order calibration
            fg = sum(v for _, v in groups_by["fetch"][i]) * scale["gather_fetch"]
            out[f"{key}:{kind}"]["fetch_bytes_gather_scale"] = round(fg)
            out[f"{key}:{kind}"]["bytes_per_launch_gather_scale"] = round(fg + wb)
    out["_calibration"] = {"kernel": f"torch neg over 2^{COPY_N.bit_length() - 1} FP32 (1 GiB read, 1 GiB written)",
                           "fetch_scale": round(scale["fetch"], 4), "write_scale": round(scale["write"], 4)}
    if "gather_fetch" in scale:
        out["_calibration"]["gather_kernel"] = ("torch index_select of 2^21 128-byte rows in random order "
                                                "(256 MiB read at random + 16 MiB indices, 256 MiB written)")
        out["_calibration"]["gather_fetch_scale"] = round(scale["gather_fetch"], 4)
        out["_calibration"]["gather_write_scale"] = round(scale.get("gather_write", float("nan")), 4)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(f"wrote {path}: {len(order)} calls; scales {scale}")


def scatter_line_bytes(kind, n, m, line=64):
    """Bytes at cache-line granularity: the sequential arrays once, and every
    line of a randomly indexed array that holds at least one target once per
    direction (m distinct random targets in n: a line of line/4 elements is
    untouched with probability (1 - m/n)^(line/4))."""
    touched = n * 4 * (1.0 - (1.0 - m / n) ** (line // 4))
    if kind == "vjp":  # is, xs_saved, vs_bar; ys_bar read + written, ys written
        return 12 * m + 3 * touched
    return 12 * m + 2 * touched  # is, vs, xs_saved; xs read + written


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
    if args.ingest_pmc:
        ingest_pmc(*args.ingest_pmc)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (sharding across GPUs is "
              "designed, not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2202_10297_amd import capi, workloads

    capi.lib()
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    L = capi.lib()
    if args.only:
        fns = {"reduce_map": bench_reduce_map, "reduce_generic": bench_reduce_generic,
               "scan_generic": bench_scan_generic, "jvp": bench_jvp, "kmeans": bench_kmeans, "gather_map": bench_gather_map,
               "scan_batched": bench_scan_batched, "sparse_kmeans": bench_sparse_kmeans, "hist_lae": bench_hist_lae,
               "hist_generic": bench_hist_generic, "scan": bench_scan,
               "gmm": bench_gmm, "batch": bench_batch, "serve": bench_serve}
        print(json.dumps({args.only: fns[args.only](args)}))
        return

    if args.copy_calibration:
        src = torch.ones(COPY_N, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
        rows = torch.ones((GATHER_ROWS, 32), dtype=torch.float32, device=dev)
        perm = torch.randperm(GATHER_ROWS, device=dev)
        out = torch.empty_like(rows)
        for _ in range(3):
            torch.index_select(rows, 0, perm, out=out)
        torch.cuda.synchronize()
        del rows, perm, out
        torch.cuda.empty_cache()

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
    vsb_s = torch.empty(M_SCAT, dtype=torch.float32, device=dev)
    plan_nb = L.pvjp_scatter_plan_bytes(capi.F32, N_SCAT, M_SCAT)
    plan = torch.empty(plan_nb, dtype=torch.uint8, device=dev)

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

    # the scatter's forward sweep returns its updates grouped by target window
    # (the plan, rebuilt every step from `is`), which the return sweep reads
    def sprim():
        capi.call("pvjp_scatter_planned", capi.F32, p(xs), N_SCAT, p(is_), p(sv), M_SCAT, p(plan), plan_nb, sp)

    def svjp():
        capi.call("pvjp_scatter_planned_vjp", capi.F32, p(ysb), N_SCAT, M_SCAT, p(vsb_s), 0, p(xs), p(plan),
                  plan_nb, sp)

    calls.append(("scatter_m2^24_n2^26", "primal", sprim, scatter_bytes(M_SCAT), M_SCAT))
    calls.append(("scatter_m2^24_n2^26", "vjp", svjp, scatter_vjp_bytes(M_SCAT), 0))
    assert [(c[0], c[1]) for c in calls] == call_order()
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

    # Parity spot check on this run's output: the + adjoint is a gather.
    it0 = inst[0]
    idx = np.random.default_rng(1).integers(0, N_HIST, 4096)
    got = it0["vsb"].cpu().numpy()[idx]
    exp = it0["hb"].cpu().numpy()[it0["ind_np"][idx]]
    if not np.array_equal(got, exp):
        log("PARITY FAILURE in the + histogram adjoint")
        sys.exit(3)
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

    # The whole step against the roofline: every call's algorithmic bytes
    # over the step's time.
    step_bytes = sum(c[3] for c in calls)
    step_roof = {"alg_bytes": step_bytes, "achieved_GBps": round(step_bytes / (ms_per_step * 1e-3) / 1e9, 1),
                 "frac": round(step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
    dom = int(np.argmax(avg))
    dkey, dkind, _, dbytes, _ = calls[dom]
    achieved = dbytes / (avg[dom] * 1e-3) / 1e9
    kernel_name = {"primal": "pvjp_hist" if dkey.startswith("hist") else "pvjp_scatter_planned",
                   "vjp": "pvjp_hist_vjp" if dkey.startswith("hist") else "pvjp_scatter_planned_vjp"}[dkind]
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
    if dkey.startswith("scatter"):
        lg = scatter_line_bytes(dkind, N_SCAT, M_SCAT)
        roof["line_granular_bytes_per_launch"] = round(lg)
        roof["frac_line_granular"] = round(lg / (avg[dom] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
    if roof["traffic"]:
        roof["traffic_GBps"] = round(roof["traffic"] / (avg[dom] * 1e-3) / 1e9, 1)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_sample, vs_np, inst, xs_np, is_np, sv_np, yb_np)
        try:
            cpu["by_config"] = oracle_by_config()
        except Exception as e:  # report, keep the main line
            cpu["by_config"] = {"error": f"{type(e).__name__}: {e}"}

    # The unplanned scatter pair (one random access per update and array) on
    # the same inputs, for comparison.
    saved = torch.empty(M_SCAT, dtype=torch.float32, device=dev)
    t_up = _events_ms(lambda: capi.call("pvjp_scatter", capi.F32, p(xs), N_SCAT, p(is_), p(sv), M_SCAT, p(saved),
                                        sp), 10)
    t_uv = _events_ms(lambda: capi.call("pvjp_scatter_vjp", capi.F32, p(ysb), N_SCAT, p(is_), M_SCAT, p(vsb_s), 0,
                                        p(xs), p(saved), sp), 10)
    detail["scatter_m2^24_n2^26"]["unplanned"] = {"primal_ms": round(t_up, 4), "vjp_ms": round(t_uv, 4)}
    del saved, plan

    # Free the histogram/scatter inputs before the other workloads.
    del inst, vs, xs, is_, sv, ysb, calls
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    extra = {}
    for name, fn in (("reduce_map", bench_reduce_map), ("reduce_generic", bench_reduce_generic),
                     ("scan_generic", bench_scan_generic), ("jvp", bench_jvp), ("kmeans", bench_kmeans),
                     ("gather_map", bench_gather_map), ("scan_batched", bench_scan_batched),
                     ("sparse_kmeans", bench_sparse_kmeans), ("hist_lae", bench_hist_lae),
                     ("hist_generic", bench_hist_generic), ("scan", bench_scan), ("gmm", bench_gmm),
                     ("batch", bench_batch), ("serve", bench_serve)):
        if name in args.skip:
            continue
        try:
            log(f"extra: {name}")
            extra[name] = fn(args)
        except Exception as e:  # report, keep the main line
            extra[name] = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

    try:
        achievable = copy_bandwidth()
    except Exception as e:  # report, keep the main line
        achievable = f"{type(e).__name__}: {e}"

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
        "step_roofline": step_roof,
        "copy_GBps_achievable": achievable,
        "cpu_baseline": cpu,
        "detail": detail,
        "other_workloads": extra,
    }
    if "serve" in extra and "p50_ms" in extra["serve"]:
        out["served_latency"] = {"p50_ms": extra["serve"]["p50_ms"], "p99_ms": extra["serve"]["p99_ms"]}
    print(json.dumps(out), flush=True)


def _events_ms(fn, reps, warm=2):
    import torch

    for _ in range(warm):
        fn()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def bench_scan(args):
    """Linear-recurrence scan, FP64: the latency-bound n = 65,536 instance and
    an HBM-bound n = 2^26 instance (primal 32 B/elem, VJP with checkpoint
    48 B/elem)."""
    import torch

    from paper_2202_10297_amd import ops, workloads

    res = {}
    for n in (65536, 1 << 26):
        a, b, ya, yb = (torch.from_numpy(x).cuda() for x in workloads.linrec(n, "f64", seed=0))
        _, _, ck = ops.linrec_scan(a, b)
        A, B = torch.empty_like(a), torch.empty_like(b)
        ab, bb = torch.empty_like(a), torch.empty_like(b)
        reps = 200 if n < 1 << 20 else 10
        tp = _events_ms(lambda: ops.linrec_scan(a, b), reps)
        tv = _events_ms(lambda: ops.linrec_scan_vjp(a, b, ya, yb, ckpt=ck, a_bar=ab, b_bar=bb), reps)
        res[f"n{n}"] = {"primal_us": round(tp * 1e3, 2), "vjp_us": round(tv * 1e3, 2),
                        "grad_over_primal": round((tp + tv) / tp, 3),
                        "vjp_elems_per_s": round(n / (tv * 1e-3), 1),
                        "primal_GBps": round(32 * n / (tp * 1e-3) / 1e9, 1),
                        "vjp_GBps": round(48 * n / (tv * 1e-3) / 1e9, 1)}
        del a, b, ya, yb, ck, A, B, ab, bb
    # C1 as 20 back-to-back calls captured in one HIP graph (outputs and
    # workspaces preallocated and zeroed before the capture; the calls go
    # straight to the C ABI on the capturing stream): kernel time without the
    # host's per-call work.
    from paper_2202_10297_amd import capi

    L = capi.lib()
    n = 65536
    a, b, ya, yb = (torch.from_numpy(x).cuda() for x in workloads.linrec(n, "f64", seed=0))
    A, B, ab, bb = (torch.empty_like(a) for _ in range(4))
    ck = torch.empty(2 * L.pvjp_linrec_ckpt_len(n), dtype=a.dtype, device=a.device)
    wf = torch.zeros(L.pvjp_linrec_scan_ws_bytes(capi.F64, n), dtype=torch.uint8, device="cuda")
    wv = torch.zeros(L.pvjp_linrec_scan_vjp_ws_bytes(capi.F64, n), dtype=torch.uint8, device="cuda")
    p_ = lambda t: t.data_ptr()

    def prim():
        capi.call("pvjp_linrec_scan", capi.F64, p_(a), p_(b), n, p_(A), p_(B), p_(ck), p_(wf), wf.numel(),
                  torch.cuda.current_stream().cuda_stream)

    def vjp():
        capi.call("pvjp_linrec_scan_vjp", capi.F64, p_(a), p_(b), p_(ya), p_(yb), n, p_(ck), p_(ab), p_(bb), 0,
                  p_(wv), wv.numel(), torch.cuda.current_stream().cuda_stream)

    prim()
    torch.cuda.synchronize()
    graphs = {}
    for name, fn in (("primal", prim), ("vjp", vjp)):
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            for _ in range(20):
                fn()
        graphs[name] = _events_ms(gr.replay, 20) / 20
    res["n65536_graph"] = {"primal_us": round(graphs["primal"] * 1e3, 2), "vjp_us": round(graphs["vjp"] * 1e3, 2),
                           "grad_over_primal": round((graphs["primal"] + graphs["vjp"]) / graphs["primal"], 3)}
    del a, b, ya, yb, ck, A, B, ab, bb, wf, wv, graphs
    torch.cuda.empty_cache()
    # C1 with the 256 MiB last-level cache flushed before every run (a 1 GiB
    # write between runs), mean and median of 20 event-timed runs.
    n = 65536
    a, b, ya, yb = (torch.from_numpy(x).cuda() for x in workloads.linrec(n, "f64", seed=0))
    _, _, ck = ops.linrec_scan(a, b)
    ab, bb = torch.empty_like(a), torch.empty_like(b)
    junk = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    tps, tvs = [], []
    for _ in range(20):
        for fn, acc in ((lambda: ops.linrec_scan(a, b), tps),
                        (lambda: ops.linrec_scan_vjp(a, b, ya, yb, ckpt=ck, a_bar=ab, b_bar=bb), tvs)):
            junk.fill_(1.0)
            s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s0.record()
            fn()
            s1.record()
            torch.cuda.synchronize()
            acc.append(s0.elapsed_time(s1) * 1e3)
    res["n65536_flushed"] = {"primal_us_mean": round(float(np.mean(tps)), 2),
                             "primal_us_median": round(float(np.median(tps)), 2),
                             "vjp_us_mean": round(float(np.mean(tvs)), 2),
                             "vjp_us_median": round(float(np.median(tvs)), 2)}
    del junk, a, b, ya, yb, ck, ab, bb
    torch.cuda.empty_cache()
    # n-sweep (FP64, a ~ U[0.5, 1), b and the adjoints ~ N(0, 1) drawn on the
    # device): where HBM starts to bind.
    sweep = {}
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    for lg in (16, 18, 20, 22, 24, 26, 28):
        n = 1 << lg
        a = torch.rand(n, dtype=torch.float64, device="cuda", generator=g) * 0.5 + 0.5
        b, ya, yb = (torch.randn(n, dtype=torch.float64, device="cuda", generator=g) for _ in range(3))
        A, B, ck = ops.linrec_scan(a, b)
        ab, bb = torch.empty_like(a), torch.empty_like(b)
        reps = 50 if lg <= 22 else 5
        tp = _events_ms(lambda: ops.linrec_scan(a, b), reps)
        tv = _events_ms(lambda: ops.linrec_scan_vjp(a, b, ya, yb, ckpt=ck, a_bar=ab, b_bar=bb), reps)
        sweep[f"2^{lg}"] = {"primal_us": round(tp * 1e3, 1), "vjp_us": round(tv * 1e3, 1),
                            "primal_hbm_frac": round(32 * n / (tp * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3),
                            "vjp_hbm_frac": round(48 * n / (tv * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3)}
        del a, b, ya, yb, A, B, ck, ab, bb
        torch.cuda.empty_cache()
    res["fp64_sweep"] = sweep
    return res


def bench_reduce_map(args):
    """reduce (+, *, max) and map (exp, tanh) primal and VJP at n = 2^26 FP32
    and FP64, inputs resident.  Algorithmic bytes: reduce reads n values
    (primal) and the VJP writes n (+, max: x_bar = y_bar or one-hot after a
    zero fill) or reads x and writes x_bar (*: p / x_i); map reads x and
    writes y (primal) and reads x, y_bar and writes x_bar (VJP)."""
    import torch

    from paper_2202_10297_amd import ops

    n = 1 << 26
    res = {}
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    for dt, tname, es in ((torch.float32, "f32", 4), (torch.float64, "f64", 8)):
        x = torch.rand(n, dtype=dt, device="cuda", generator=g) * 1.5 + 0.5  # in [0.5, 2): products stay finite
        sign = torch.where(torch.rand(n, device="cuda", generator=g) < 0.5, -1.0, 1.0).to(dt)
        x = x * sign
        xb = torch.empty_like(x)
        for op, vjp_bytes in (("add", es), ("mul", 2 * es), ("max", es)):
            y, aux = ops.reduce(op, x)
            yb = torch.ones_like(y)
            tp = _events_ms(lambda: ops.reduce(op, x), 10)
            tv = _events_ms(lambda: ops.reduce_vjp(op, x, aux, yb, x_bar=xb), 10)
            res[f"reduce_{op}_{tname}"] = {
                "primal_ms": round(tp, 4), "vjp_ms": round(tv, 4), "grad_over_primal": round((tp + tv) / tp, 3),
                "primal_hbm_frac": round(es * n / (tp * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3),
                "vjp_hbm_frac": round(vjp_bytes * n / (tv * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3)}
        ybar = torch.randn(n, dtype=dt, device="cuda", generator=g)
        xa = x.abs()
        for fn in ("exp", "tanh"):
            tp = _events_ms(lambda: ops.map_(fn, xa), 10)
            tv = _events_ms(lambda: ops.map_vjp(fn, xa, ybar, x_bar=xb), 10)
            res[f"map_{fn}_{tname}"] = {
                "primal_ms": round(tp, 4), "vjp_ms": round(tv, 4), "grad_over_primal": round((tp + tv) / tp, 3),
                "primal_hbm_frac": round(2 * es * n / (tp * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3),
                "vjp_hbm_frac": round(3 * es * n / (tv * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3)}
        del x, xb, sign, ybar, xa
        torch.cuda.empty_cache()
    # The write-only adjoints again at 2^28 FP32 (1 GiB written, four times
    # the 256 MiB last-level cache, which a 2^26 stream could partly live in).
    from paper_2202_10297_amd import capi

    n2 = 1 << 28
    x = torch.rand(n2, dtype=torch.float32, device="cuda", generator=g)
    xb = torch.empty_like(x)
    wo = {}
    for op in ("add", "max"):
        y, aux = ops.reduce(op, x)
        yb = torch.ones_like(y)
        tv = _events_ms(lambda: ops.reduce_vjp(op, x, aux, yb, x_bar=xb), 10)
        wo[f"reduce_{op}_vjp"] = {"ms": round(tv, 4), "hbm_frac": round(4 * n2 / (tv * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3)}
    m = 1 << 16
    winner = (torch.arange(m, device="cuda", dtype=torch.int32) * (n2 // m)).contiguous()
    hb = torch.ones(m, dtype=torch.float32, device="cuda")
    sp = torch.cuda.current_stream().cuda_stream
    tv = _events_ms(lambda: capi.call("pvjp_hist_vjp", capi.MAX, capi.F32, None, None, n2, m, winner.data_ptr(), None,
                                      None, hb.data_ptr(), xb.data_ptr(), 0, sp), 10)
    wo["hist_max_vjp_m65536"] = {"ms": round(tv, 4),
                                 "hbm_frac": round((4 * n2 + 12 * m) / (tv * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3)}
    res["write_only_fp32_2^28"] = wo
    del x, xb, winner, hb
    torch.cuda.empty_cache()
    return res


def bench_reduce_generic(args):
    """reduce with a general operator (Sec. 5.1.1, general rule) and its VJP
    at n = 2^26 elements, inputs resident: log-add-exp (K = 1), the linear
    recurrence (K = 2) and the 2x2 matrix product (K = 4).  Algorithmic bytes:
    the primal reads the n K components; the VJP reads them and writes their
    adjoints (2 n K per element size).  The kernels move 3 n K (x is read
    twice: tile folds, then prefixes/suffixes and f); the rule as the paper
    states it, two whole-array scans plus a map, needs at least 5.  With the
    per-tile checkpoint of the primal (32 bytes per tile) the VJP moves the
    algorithmic 2 n K."""
    import torch

    from paper_2202_10297_amd import ops

    n = 1 << 26
    res = {}
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    for op, K in (("logaddexp", 1), ("linrec", 2), ("mat2", 4)):
        for dt, tname, es in ((torch.float32, "f32", 4), (torch.float64, "f64", 8)):
            if op == "logaddexp":
                xs = [torch.randn(n, dtype=dt, device="cuda", generator=g)]
            elif op == "linrec":
                xs = [torch.rand(n, dtype=dt, device="cuda", generator=g) * 0.5 + 0.5,
                      torch.randn(n, dtype=dt, device="cuda", generator=g)]
            else:  # rotations, each composed with diag(1, -1) with probability 1/2
                th = (torch.rand(n, dtype=dt, device="cuda", generator=g) * 2 - 1) * 3.141592653589793
                f = torch.where(torch.rand(n, device="cuda", generator=g) < 0.5, -1.0, 1.0).to(dt)
                c, s_ = torch.cos(th), torch.sin(th)
                xs = [c, -s_ * f, s_, c * f]
                del th, f
            yb = [torch.randn(1, dtype=dt, device="cuda", generator=g) for _ in range(K)]
            xb = [torch.empty_like(x) for x in xs]
            tp = _events_ms(lambda: ops.reduce_generic(op, xs), 10)
            tv = _events_ms(lambda: ops.reduce_generic_vjp(op, xs, yb, x_bar=xb), 10)
            _, ck = ops.reduce_generic(op, xs, ckpt=True)
            tpc = _events_ms(lambda: ops.reduce_generic(op, xs, ckpt=True), 10)
            tvc = _events_ms(lambda: ops.reduce_generic_vjp(op, xs, yb, x_bar=xb, ckpt=ck), 10)
            comp = n * K * es
            res[f"{op}_{tname}"] = {
                "primal_ms": round(tp, 4), "vjp_ms": round(tv, 4), "grad_over_primal": round((tp + tv) / tp, 3),
                "primal_hbm_frac": round(comp / (tp * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3),
                "vjp_hbm_frac_algorithmic": round(2 * comp / (tv * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3),
                "vjp_hbm_frac_moved": round(3 * comp / (tv * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3),
                "vjp_elems_per_s": round(n / (tv * 1e-3), 1),
                "with_tile_ckpt": {
                    "primal_ms": round(tpc, 4), "vjp_ms": round(tvc, 4),
                    "grad_over_primal": round((tpc + tvc) / tpc, 3),
                    "vjp_hbm_frac": round(2 * comp / (tvc * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3)}}
            del xs, xb, yb, ck
            torch.cuda.empty_cache()
    return res


def _gop_inputs(op, n, dt, g):
    import torch

    if op == "logaddexp":
        return [torch.randn(n, dtype=dt, device="cuda", generator=g)]
    if op == "linrec":
        return [torch.rand(n, dtype=dt, device="cuda", generator=g) * 0.5 + 0.5,
                torch.randn(n, dtype=dt, device="cuda", generator=g)]
    # rotations, each composed with diag(1, -1) with probability 1/2
    th = (torch.rand(n, dtype=dt, device="cuda", generator=g) * 2 - 1) * 3.141592653589793
    f = torch.where(torch.rand(n, device="cuda", generator=g) < 0.5, -1.0, 1.0).to(dt)
    c, s_ = torch.cos(th), torch.sin(th)
    return [c, -s_ * f, s_, c * f]


def bench_scan_generic(args):
    """Inclusive scan with a general operator and its VJP by the d x d
    Jacobian rule (Sec. 5.2) at n = 2^26, with the per-tile checkpoint.
    Algorithmic bytes: the primal reads x and writes y (2 n K per element
    size), the VJP reads x and y_bar and writes x_bar (3 n K).  Moved: x is
    read twice by the primal (tile folds, then the scan) and x and y_bar twice
    by the VJP (lin_o tile folds, then the adjoints): 3 n K and 5 n K."""
    import torch

    from paper_2202_10297_amd import ops

    n = 1 << 26
    res = {}
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    for op, K in (("logaddexp", 1), ("linrec", 2), ("mat2", 4)):
        for dt, tname, es in ((torch.float32, "f32", 4), (torch.float64, "f64", 8)):
            xs = _gop_inputs(op, n, dt, g)
            yb = [torch.randn(n, dtype=dt, device="cuda", generator=g) for _ in range(K)]
            xb = [torch.empty_like(x) for x in xs]
            _, ck = ops.scan_generic(op, xs)
            tp = _events_ms(lambda: ops.scan_generic(op, xs), 5)
            tv = _events_ms(lambda: ops.scan_generic_vjp(op, xs, yb, x_bar=xb, ckpt=ck), 5)
            comp = n * K * es
            res[f"{op}_{tname}"] = {
                "primal_ms": round(tp, 4), "vjp_ms": round(tv, 4), "grad_over_primal": round((tp + tv) / tp, 3),
                "primal_hbm_frac": round(2 * comp / (tp * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3),
                "primal_hbm_frac_moved": round(3 * comp / (tp * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3),
                "vjp_hbm_frac": round(3 * comp / (tv * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3),
                "vjp_hbm_frac_moved": round(5 * comp / (tv * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3),
                "vjp_elems_per_s": round(n / (tv * 1e-3), 1)}
            del xs, xb, yb, ck
            torch.cuda.empty_cache()
    return res


def bench_scan_batched(args):
    """The regular segmented scan (a vectorised operator's scan): B = 1024
    rows of L = 65536 (2^26 elements, as the single scan above), with the
    per-tile checkpoint; the same algorithmic and moved bytes per element."""
    import torch

    from paper_2202_10297_amd import ops

    B, L = 1024, 1 << 16
    n = B * L
    res = {}
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    for op, K, dt, tname, es in (("logaddexp", 1, torch.float32, "f32", 4), ("linrec", 2, torch.float64, "f64", 8),
                                 ("mat2", 4, torch.float32, "f32", 4)):
        xs = [x.view(B, L) for x in _gop_inputs(op, n, dt, g)]
        yb = [torch.randn(B, L, dtype=dt, device="cuda", generator=g) for _ in range(K)]
        xb = [torch.empty_like(x) for x in xs]
        _, ck = ops.scan_generic_batched(op, xs)
        tp = _events_ms(lambda: ops.scan_generic_batched(op, xs), 5)
        tv = _events_ms(lambda: ops.scan_generic_batched_vjp(op, xs, yb, x_bar=xb, ckpt=ck), 5)
        comp = n * K * es
        res[f"{op}_{tname}"] = {
            "primal_ms": round(tp, 4), "vjp_ms": round(tv, 4), "grad_over_primal": round((tp + tv) / tp, 3),
            "primal_hbm_frac": round(2 * comp / (tp * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3),
            "vjp_hbm_frac": round(3 * comp / (tv * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3)}
        del xs, xb, yb, ck
        torch.cuda.empty_cache()
    return res


def bench_sparse_kmeans(args):
    """Sparse k-means (k = 10) on bag-of-words-like CSR points shaped like the
    paper's largest text workload's vocabulary: 100000 rows x 102660
    columns, about 230 distinct entries per row (Zipf(1.1) columns).  The
    objective, the gradient, and the gradient with the Hessian diagonal."""
    import torch

    from paper_2202_10297_amd import ops, workloads

    N, D, K = 100000, 102660, 10
    rp, cl, v, C = workloads.sparse_kmeans(N, D, K, 330.0, "f32", seed=0)
    drp, dcl, dv, dC = (torch.from_numpy(a).cuda() for a in (rp, cl, v, C))
    _, a = ops.sparse_kmeans_objective(drp, dcl, dv, D, dC)
    ones = torch.ones_like(dC)
    out = (torch.empty_like(dC), torch.empty_like(dC))
    tf = _events_ms(lambda: ops.sparse_kmeans_objective(drp, dcl, dv, D, dC), 10)
    tg = _events_ms(lambda: ops.sparse_kmeans_vjp(drp, dcl, dv, D, dC, a, out=(out[0], None)), 10)
    th = _events_ms(lambda: ops.sparse_kmeans_vjp(drp, dcl, dv, D, dC, a, C_dot=ones, out=out), 10)
    nnz = int(rp[-1])
    return {"rows": N, "cols": D, "k": K, "nnz": nnz, "objective_ms": round(tf, 4), "gradient_ms": round(tg, 4),
            "gradient_and_hessian_diag_ms": round(th, 4), "newton_step_ms": round(tf + th, 4),
            "objective_nnz_per_s": round(nnz / (tf * 1e-3), 1)}


def bench_hist_lae(args):
    """reduce_by_index with the log-add-exp operator at n = 2^26 FP32, m =
    2^16 and 2^20 bins, Zipf(1.1) indices.  Algorithmic bytes: primal 8 per
    element (indices, values) + 4 per bin; VJP 12 per element (indices,
    values read, adjoints written) + 8 per bin (hs, hs_bar)."""
    import torch

    from paper_2202_10297_amd import ops, workloads

    n = 1 << 26
    res = {}
    for m in (1 << 16, 1 << 20):
        inds, x, hb = (torch.from_numpy(a).cuda() for a in workloads.hist(n, m, "zipf", "f32", seed=0))
        hs = ops.hist_lae(inds, x, m)
        xb = torch.empty_like(x)
        tp = _events_ms(lambda: ops.hist_lae(inds, x, m), 10)
        tv = _events_ms(lambda: ops.hist_lae_vjp(inds, x, hs, hb, x_bar=xb), 10)
        res[f"m2^{m.bit_length() - 1}_zipf"] = {
            "primal_ms": round(tp, 4), "vjp_ms": round(tv, 4), "grad_over_primal": round((tp + tv) / tp, 3),
            "primal_hbm_frac": round((8 * n + 4 * m) / (tp * 1e-3) / 8e12, 3),
            "vjp_hbm_frac": round((12 * n + 8 * m) / (tv * 1e-3) / 8e12, 3)}
        del inds, x, hb, hs, xb
    return res


def bench_hist_generic(args):
    """reduce_by_index with a general, non-commuting operator (the linear
    recurrence, K = 2, and the 2x2 matrix product, K = 4) at n = 2^26 FP32,
    m = 2^16 bins, uniform indices: stable sort by bin, segmented scans.
    Algorithmic bytes: primal 4 + 4 K per element + 4 K per bin; VJP 4 + 8 K
    per element (indices and x read, x_bar written) + 4 K per bin."""
    import torch

    from paper_2202_10297_amd import ops, workloads

    n, m = 1 << 26, 1 << 16
    res = {}
    for op in ("linrec", "mat2"):
        inds, xs, hb = workloads.hist_generic(op, n, m, "uniform", "f32", seed=0)
        di = torch.from_numpy(inds).cuda()
        dx = [torch.from_numpy(x).cuda() for x in xs]
        dh = [torch.from_numpy(h).cuda() for h in hb]
        del inds, xs, hb
        K = len(dx)
        ops.hist_generic(op, di, dx, m)
        xb = [torch.empty_like(x) for x in dx]
        tp = _events_ms(lambda: ops.hist_generic(op, di, dx, m), 5)
        tv = _events_ms(lambda: ops.hist_generic_vjp(op, di, dx, dh, x_bar=xb), 5)
        res[f"{op}_m2^16_uniform"] = {
            "primal_ms": round(tp, 3), "vjp_ms": round(tv, 3), "grad_over_primal": round((tp + tv) / tp, 3),
            "primal_elems_per_s": round(n / (tp * 1e-3), 1), "vjp_elems_per_s": round(n / (tv * 1e-3), 1),
            "primal_hbm_frac": round(((4 + 4 * K) * n + 4 * K * m) / (tp * 1e-3) / 8e12, 4),
            "vjp_hbm_frac": round(((4 + 8 * K) * n + 4 * K * m) / (tv * 1e-3) / 8e12, 4)}
        del di, dx, dh, xb
        torch.cuda.empty_cache()
    return res


def bench_jvp(args):
    """Forward mode at n = 2^26 (tangents resident): map (exp), reduce(+),
    reduce_by_index (+ at m = 2^16 Zipf, max at m = 2^20), scatter (2^24
    targets into 2^26) and the general-operator reduce and scan on (x, x_dot)
    pairs.  Algorithmic bytes: map 3 s n (x, x_dot read, y_dot written);
    reduce 4 n; histogram + 8 n, max 12 m; scatter 12 m; general reduce
    2 K s n; general scan 4 K s n (x, x_dot read, y, y_dot written)."""
    import torch

    from paper_2202_10297_amd import ops, workloads

    n = 1 << 26
    res = {}
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    rate = lambda b, t: round(b / (t * 1e-3) / 1e9 / HBM_PEAK_GBPS, 3)
    x = torch.rand(n, device="cuda", generator=g) + 0.5
    xd = torch.randn(n, device="cuda", generator=g)
    t = _events_ms(lambda: ops.map_jvp("exp", x, xd), 10)
    res["map_exp_f32"] = {"ms": round(t, 4), "hbm_frac": rate(12 * n, t)}
    _, aux = ops.reduce("add", x)
    t = _events_ms(lambda: ops.reduce_jvp("add", x, aux, xd), 10)
    res["reduce_add_f32"] = {"ms": round(t, 4), "hbm_frac": rate(4 * n, t)}
    for op, m, dist in (("add", 1 << 16, "zipf"), ("max", 1 << 20, "uniform")):
        inds, vs, _ = workloads.hist(n, m, dist, "f32", seed=0)
        di, dv = torch.from_numpy(inds).cuda(), torch.from_numpy(vs).cuda()
        _, aux = ops.hist(op, di, dv, m)
        t = _events_ms(lambda: ops.hist_jvp(op, di, xd, m, aux), 10)
        res[f"hist_{op}_m{m}_f32"] = {"ms": round(t, 4),
                                     "hbm_frac": rate(8 * n if op == "add" else 12 * m, t)}
        del di, dv
    m = 1 << 24
    is_ = torch.randperm(n, device="cuda", generator=g)[:m].to(torch.int32)
    vd = torch.randn(m, device="cuda", generator=g)
    yd = xd.clone()
    t = _events_ms(lambda: ops.scatter_jvp_(yd, is_, vd), 10)
    res["scatter_f32"] = {"ms": round(t, 4), "hbm_frac": rate(12 * m, t)}
    del x, xd, is_, vd, yd
    torch.cuda.empty_cache()
    for op, K in (("logaddexp", 1), ("linrec", 2)):
        for dt, tname, es in ((torch.float32, "f32", 4), (torch.float64, "f64", 8)):
            xs = _gop_inputs(op, n, dt, g)
            xds = [torch.randn(n, dtype=dt, device="cuda", generator=g) for _ in range(K)]
            tr = _events_ms(lambda: ops.reduce_generic_jvp(op, xs, xds), 5)
            ts = _events_ms(lambda: ops.scan_generic_jvp(op, xs, xds), 5)
            res[f"{op}_{tname}"] = {"reduce_ms": round(tr, 4), "reduce_hbm_frac": rate(2 * K * es * n, tr),
                                    "scan_ms": round(ts, 4), "scan_hbm_frac": rate(4 * K * es * n, ts)}
            del xs, xds
            torch.cuda.empty_cache()
    return res


def bench_kmeans(args):
    """Dense k-means at the paper's shapes (k, n, d) = (5, 494019, 35) and
    (1024, 10000, 256): the objective (nearest-centre search, FP64 distance
    chains), the gradient from the kept assignments, and the gradient with the
    jvp of the VJP (Hessian diagonal) in the same pass.  The search does
    n k d FP64 FMAs."""
    import torch

    from paper_2202_10297_amd import ops, workloads

    res = {}
    for K, N, D in ((5, 494019, 35), (1024, 10000, 256)):
        X, C = workloads.kmeans(N, D, K, "f32", seed=0)
        Xd, Cd = torch.from_numpy(X).cuda(), torch.from_numpy(C).cuda()
        _, a = ops.kmeans_objective(Xd, Cd)
        ones = torch.ones_like(Cd)
        out = (torch.empty_like(Cd), torch.empty_like(Cd))
        tf = _events_ms(lambda: ops.kmeans_objective(Xd, Cd), 10)
        tg = _events_ms(lambda: ops.kmeans_vjp(Xd, Cd, a, out=(out[0], None)), 10)
        th = _events_ms(lambda: ops.kmeans_vjp(Xd, Cd, a, C_dot=ones, out=out), 10)
        res[f"k{K}_n{N}_d{D}"] = {
            "objective_ms": round(tf, 4), "gradient_ms": round(tg, 4), "gradient_and_hessian_diag_ms": round(th, 4),
            "search_fp64_TFLOPs": round(2 * N * K * D / (tf * 1e-3) / 1e12, 2),
            "newton_step_ms": round(tf + th, 4)}
    return res


def bench_gather_map(args):
    """A map reading a free array at 2^26 computed indices (FP32, a v): the
    primal and the return sweep with the reads accumulated into as_bar, for
    n = 2^12 (LDS bins) and 2^20 (global atomics), Zipf(1.1) and uniform
    indices.  Algorithmic bytes: primal 12 B per element (is, vs read, ys
    written); VJP 16 B (is, vs, ys_bar read, vs_bar written) + 8 n (as
    read, as_bar written)."""
    import torch

    from paper_2202_10297_amd import ops, workloads

    m = 1 << 26
    res = {}
    for n, dist in ((1 << 12, "zipf"), (1 << 12, "uniform"), (1 << 20, "zipf"), (1 << 20, "uniform")):
        as_, is_, vs, yb = (torch.from_numpy(a).cuda() for a in workloads.gather_map(m, n, dist, "f32", seed=0))
        ys = torch.empty(m, dtype=torch.float32, device="cuda")
        ab = torch.empty(n, dtype=torch.float32, device="cuda")
        vb = torch.empty(m, dtype=torch.float32, device="cuda")
        tp = _events_ms(lambda: ops.gather_map("mul", as_, is_, vs, out=ys), 10)
        tv = _events_ms(lambda: ops.gather_map_vjp("mul", as_, is_, vs, yb, as_bar=ab, vs_bar=vb), 10)
        res[f"n2^{n.bit_length() - 1}_{dist}"] = {
            "primal_ms": round(tp, 4), "vjp_ms": round(tv, 4), "grad_over_primal": round((tp + tv) / tp, 3),
            "primal_hbm_frac": round(12 * m / (tp * 1e-3) / 8e12, 3),
            "vjp_hbm_frac": round((16 * m + 8 * n) / (tv * 1e-3) / 8e12, 3)}
        del as_, is_, vs, yb, ys, ab, vb
    return res


def copy_bandwidth():
    """Device-to-device copy of 1 GiB (read + write counted): the achievable
    HBM rate beside the 8 TB/s datasheet peak."""
    import torch

    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    t = _events_ms(lambda: dst.copy_(src), 10)
    del src, dst
    torch.cuda.empty_cache()
    return round(2 * (1 << 30) / (t * 1e-3) / 1e9, 1)


def bench_gmm(args):
    """GMM N = 10^6, D = 64, K = 200 (FP32, FP64 LSE): objective and gradient.
    Algorithmic flops: forward N K D (D+1) with the triangle of Q_k used,
    gradient about twice that (recomputation + the contraction of G_k); with
    the s_ik checkpoint the gradient is one contraction, N K D (D+1)."""
    import torch

    from paper_2202_10297_amd import ops, workloads

    N, D, K = 1_000_000, 64, 200
    P = [torch.from_numpy(x).cuda() for x in workloads.gmm(N, D, K, seed=0)]
    _, lse = ops.gmm_objective(*P)
    tf = _events_ms(lambda: ops.gmm_objective(*P), 5)
    out = tuple(torch.empty_like(t) for t in P[1:])
    tb = _events_ms(lambda: ops.gmm_vjp(*P, lse=lse, out=out), 5)
    # with the s_ik checkpoint (8 N K bytes): one contraction in the gradient
    sck = torch.empty((K, N), dtype=torch.float64, device="cuda")
    _, lse2 = ops.gmm_objective(*P, s_out=sck)
    tfs = _events_ms(lambda: ops.gmm_objective(*P, s_out=sck), 5)
    tbs = _events_ms(lambda: ops.gmm_vjp(*P, lse=lse2, s=sck, out=out), 5)
    del sck
    flop_f = N * K * D * (D + 1)
    return {"objective_ms": round(tf, 3), "gradient_ms": round(tb, 3), "grad_over_primal": round((tf + tb) / tf, 3),
            "objective_TFLOPs": round(flop_f / (tf * 1e-3) / 1e12, 1),
            "gradient_TFLOPs": round(2 * flop_f / (tb * 1e-3) / 1e12, 1),
            "vjp_points_per_s": round(N / (tb * 1e-3), 1),
            "with_s_ckpt": {"objective_ms": round(tfs, 3), "gradient_ms": round(tbs, 3),
                            "grad_over_primal": round((tfs + tbs) / tfs, 3),
                            "gradient_TFLOPs": round(flop_f / (tbs * 1e-3) / 1e12, 1),
                            "ckpt_bytes": 8 * N * K}}


def bench_batch(args):
    """4,096 scan VJPs + 4,096 sum-reduce VJPs, lengths log-uniform in
    [64, 2^20], FP32: one persistent launch (autotuned tile and grid, replayed
    from a HIP graph) against one launch per instance."""
    import torch

    from paper_2202_10297_amd import batch, ops, workloads

    lengths = workloads.segment_lengths(4096, 64, 1 << 20, seed=0)
    total = int(lengths.sum())
    g = workloads.rng(0)
    dev = torch.device("cuda")
    a = torch.from_numpy(g.uniform(0.5, 1.0, total).astype(np.float32)).to(dev)
    b = torch.from_numpy(g.standard_normal(total, dtype=np.float32)).to(dev)
    ya = torch.from_numpy(g.standard_normal(total, dtype=np.float32)).to(dev)
    yb = torch.from_numpy(g.standard_normal(total, dtype=np.float32)).to(dev)
    sy = torch.from_numpy(g.standard_normal(4096).astype(np.float32)).to(dev)
    ab, bb, sx = torch.empty_like(a), torch.empty_like(a), torch.empty_like(a)
    t0 = time.time()
    probe = batch.SegPlan(lengths, torch.float32)
    _, _, ck0 = probe.scan(a, b, outputs=False)
    tile, grid = __import__("paper_2202_10297_amd.tune", fromlist=["x"]).seg_config(
        probe, dict(a=a, b=b, yA_bar=ya, yB_bar=yb, a_bar=ab, b_bar=bb, sum_ybar=sy, sum_xbar=sx))
    tune_s = time.time() - t0
    plan = batch.SegPlan(lengths, torch.float32, tile=tile, grid=grid)
    _, _, ck = plan.scan(a, b, outputs=False)
    kw = dict(a=a, b=b, yA_bar=ya, yB_bar=yb, ckpt=ck, a_bar=ab, b_bar=bb, sum_ybar=sy, sum_xbar=sx)
    t_eager = _events_ms(lambda: plan.vjp(**kw), 5)
    plan.capture(**kw)
    t_graph = _events_ms(plan.replay, 5)
    # one launch per instance
    off = plan.offsets
    cks = []
    for s in range(4096):
        lo, hi = int(off[s]), int(off[s + 1])
        cks.append(ops.linrec_scan(a[lo:hi], b[lo:hi])[2])
    aux = {}

    def per_instance():
        for s in range(4096):
            lo, hi = int(off[s]), int(off[s + 1])
            ops.linrec_scan_vjp(a[lo:hi], b[lo:hi], ya[lo:hi], yb[lo:hi], ckpt=cks[s], a_bar=ab[lo:hi],
                                b_bar=bb[lo:hi])
            ops.reduce_vjp("add", a[lo:hi], aux, sy[s:s + 1], x_bar=sx[lo:hi])

    t_each = _events_ms(per_instance, 2, warm=1)
    alg = 24 * total + 4 * total
    return {"segments": 4096, "elements_per_set": total, "tile_elems": tile, "grid_blocks": grid,
            "tune_s": round(tune_s, 2), "batched_ms": round(t_eager, 3), "graph_replay_ms": round(t_graph, 3),
            "per_instance_ms": round(t_each, 3), "speedup_vs_per_instance": round(t_each / t_graph, 2),
            "alg_GBps": round(alg / (t_graph * 1e-3) / 1e9, 1),
            "vjp_elems_per_s": round(2 * total / (t_graph * 1e-3), 1)}


def bench_serve(args):
    """Poisson arrivals at 2,000 requests/s for 30 s after a 5 s warm-up,
    mixing scan VJPs (n in [1e3, 1e7]), + histogram VJPs (n in [1e4, 1e7],
    2^12..2^18 bins, Zipf) and GMM gradients (N in [1e3, 1e5], D = 32,
    K = 50) over 256 resident instances per kind under a 64 GB budget; the
    same trace served serially (one slot) for comparison; then a saturating
    burst (every request arriving at once) served both ways, whose throughput
    shows what overlapping requests on the device buys."""
    from paper_2202_10297_amd import serve

    t0 = time.time()
    pool = serve.Pool(per_kind=256, seed=0, device_gen=True)
    build_s = time.time() - t0
    warm = 5.0
    keep = lambda d: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}
    out = {}
    for slots, name in ((8, None), (1, "serial_one_slot")):
        trace = serve.make_trace(pool, rate=2000.0, duration=warm + args.serve_seconds, seed=0)
        log(f"serve: {slots} slot(s), {len(trace)} requests")
        st, _ = serve.Server(pool, slots=slots, budget_bytes=64 << 30).run(trace, warmup=warm)
        if name is None:
            out = keep(st)
        else:
            out[name] = keep({k: st[k] for k in ("p50_ms", "p99_ms", "throughput_rps", "max_inflight")})
    sat = {}
    for slots in (8, 1):
        burst = serve.make_burst(pool, 1500, seed=1)
        st, _ = serve.Server(pool, slots=slots, budget_bytes=64 << 30).run(burst)
        sat[f"slots{slots}"] = keep({k: st[k] for k in ("throughput_rps", "elems_per_s", "p50_ms", "p99_ms",
                                                         "max_inflight", "wall_s")})
    out["saturation_burst_1500"] = sat
    out["rate_rps"] = 2000.0
    out["warmup_s"] = warm
    out["measured_s"] = args.serve_seconds
    out["resident_per_kind"] = 256
    out["pool_build_s"] = round(build_s, 1)
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def _host_threads():
    """Threads for the oracle's P-thread baselines: the host's cores, capped at
    16 (one GPU's share of a box's CPUs)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _threaded(jobs, threads, prepare=None):
    """Runs the callables in `jobs` on `threads` host threads (the oracle's C
    calls release the GIL) and returns the wall time.  With `prepare`, job i
    is called with prepare[i]()'s result, and the preparation (input
    generation) runs on the same threads before the timed region."""
    import concurrent.futures as cf

    with cf.ThreadPoolExecutor(threads) as ex:
        args = [f.result() for f in [ex.submit(pr) for pr in prepare]] if prepare else [None] * len(jobs)
        t0 = time.perf_counter()
        for f in [ex.submit(j, *(() if a is None else (a,))) for j, a in zip(jobs, args)]:
            f.result()
        return time.perf_counter() - t0


def oracle_by_config(serve_pool_seed=0):
    """The oracle timed on this host for the other configurations, on bounded
    samples (each a few seconds of CPU work), as SURVEY-style baselines:
      C1  the n = 65,536 FP64 scan, primal + taped VJP, one thread, full size;
      C3  GMM (D = 64, K = 200) objective + taped gradient on a sample of
          points, P threads over point chunks and one thread;
      C4  scan VJPs + sum VJPs over the first segments of the batch's length
          table, P threads over segments;
      C5  the first requests of the serving trace, offline, P threads.
    Rates are measured on the sample, never extrapolated."""
    sys.path.insert(0, ROOT)
    import oracle
    from paper_2202_10297_amd import workloads

    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    P = _host_threads()
    res = {"threads": P, "host_cores": os.cpu_count(), "cpu_model": _cpu_model()}
    # C1
    a, b, ya, yb = workloads.linrec(65536, "f64", seed=0)
    reps, t0 = 0, time.perf_counter()
    while reps < 3 or time.perf_counter() - t0 < 1.0:
        oracle.linrec_scan(a, b)
        oracle.linrec_scan_vjp(a, b, ya, yb)
        reps += 1
    dt = (time.perf_counter() - t0) / reps
    res["C1"] = {"value": round(65536 / dt, 1), "unit": "VJP elems/s (primal + taped VJP)", "cores": 1,
                 "ms_per_instance": round(dt * 1e3, 3), "sample": "the full n = 65,536 FP64 instance", "reps": reps}
    # C3
    per = 40
    X, al, mu, q, l = workloads.gmm(P * per, 64, 200, seed=0)

    def gmm_job(lo, hi):
        return lambda: (oracle.gmm_objective(X[lo:hi], al, mu, q, l), oracle.gmm_vjp(X[lo:hi], al, mu, q, l, 1.0))

    wall = _threaded([gmm_job(i * per, (i + 1) * per) for i in range(P)], P)
    t1 = time.perf_counter()
    gmm_job(0, 100)()
    one = time.perf_counter() - t1
    res["C3"] = {"value": round(P * per / wall, 2), "unit": "points/s (objective + taped gradient)", "cores": P,
                 "sample": f"{P * per} points of N = 10^6 (D = 64, K = 200), {per} per thread",
                 "one_thread": {"value": round(100 / one, 2), "cores": 1, "sample": "100 points"}}
    # C4
    lengths = workloads.segment_lengths(4096, 64, 1 << 20, seed=0)
    cut = int(np.searchsorted(np.cumsum(lengths), 1 << 24)) + 1
    segs = [int(L) for L in lengths[:cut]]

    def seg_inputs(L, s):
        def prep():
            gg = workloads.rng(100 + s)
            return (gg.uniform(0.5, 1.0, L), gg.standard_normal(L), gg.standard_normal(L), gg.standard_normal(L))
        return prep

    def seg_run(x):
        oracle.linrec_scan_vjp(*x)
        oracle.reduce_vjp("add", x[1], 1.0)

    wall = _threaded([seg_run] * len(segs), P, prepare=[seg_inputs(L, s) for s, L in enumerate(segs)])
    tot = sum(segs)
    res["C4"] = {"value": round(2 * tot / wall, 1), "unit": "VJP elems/s (scan + sum)", "cores": P,
                 "sample": f"the first {len(segs)} of 4,096 segments ({tot} elements per set)"}
    # C5
    try:
        res["C5"] = _oracle_serve_offline(oracle, workloads, P, nreq=8)
    except Exception as e:  # report, keep the rest
        res["C5"] = {"error": f"{type(e).__name__}: {e}"}
    return res


def _oracle_serve_offline(oracle, workloads, P, nreq):
    """The first `nreq` requests of the serving trace (same pool seeds and
    sizes as the served run), evaluated by the oracle on P threads."""
    g = workloads.rng(0)
    logu = lambda lo, hi: int(np.exp(g.uniform(np.log(lo), np.log(hi))))
    per_kind = 24
    spec = {"scan": [logu(1e3, 1e7) for _ in range(per_kind)]}
    spec["hist"] = []
    for _ in range(per_kind):
        n = logu(1e4, 1e7)
        spec["hist"].append((n, 1 << int(g.integers(12, 19))))
    spec["gmm"] = [logu(1e3, 1e5) for _ in range(per_kind)]
    gt = workloads.rng(12345)
    n_arr = int(2000.0 * 5.0 * 1.2) + 16
    t = np.cumsum(gt.exponential(1.0 / 2000.0, n_arr))
    kinds = gt.choice(3, size=t.size, p=np.full(3, 1 / 3))
    prep, jobs, elems, names = [], [], 0, []
    for k in kinds[:nreq]:
        kind = ("scan", "hist", "gmm")[int(k)]
        i = int(gt.integers(0, per_kind))
        v = int(gt.integers(0, 2))
        names.append(kind)
        if kind == "scan":
            n = spec["scan"][i]
            elems += n
            prep.append(lambda n=n, i=i, v=v: (*workloads.linrec(n, "f32", seed=i)[:2],
                                               *workloads.linrec(n, "f32", seed=i + 7919 * (v + 1))[2:]))
            jobs.append(lambda x: oracle.linrec_scan_vjp(*x))
        elif kind == "hist":
            n, m = spec["hist"][i]
            elems += n
            prep.append(lambda n=n, m=m, i=i, v=v: (workloads.hist(n, m, "zipf", "f32", seed=i)[0], np.zeros(n),
                                                    workloads.rng(i + 31 * (v + 1)).standard_normal(m)))
            jobs.append(lambda x: oracle.hist_vjp("add", *x))
        else:
            N = spec["gmm"][i]
            elems += N
            prep.append(lambda N=N, i=i, v=v: (workloads.gmm(N, 32, 50, seed=3000 * 0 + i), 1.0 + 0.5 * v))
            jobs.append(lambda x: oracle.gmm_vjp(*x[0], x[1]))
    wall = _threaded(jobs, P, prepare=prep)
    return {"value": round(nreq / wall, 3), "unit": "requests/s (offline)", "cores": min(P, nreq),
            "sample": f"the first {nreq} requests of the 2,000 req/s trace ({', '.join(names)})", "elements": elems}


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
    host = [(it["inds"][:ns].cpu().numpy(), it["hb"].cpu().numpy()) for it in inst]  # outside the timing
    t0 = time.perf_counter()
    for it, (ind, hb) in zip(inst, host):
        oracle.hist(it["op"], ind, vsn, it["m"])
        oracle.hist_vjp(it["op"], ind, vsn, hb)
        elems += ns
    sel = is_np[is_np < ns][: ns // 4]
    oracle.scatter(xs_np[:ns], sel, sv_np[: sel.size])
    oracle.scatter_vjp(sel, yb_np[:ns])
    elems += sel.size
    dt = time.perf_counter() - t0
    model = _cpu_model()
    return {
        "value": round(elems / dt, 1),
        "unit": "elems/s",
        "cores": 1,
        "host_cores": os.cpu_count(),
        "cpu_model": model,
        "kind": "oracle",
        "sample": f"first {ns} elements of each of the 12 histogram instances (+ and max, primal and taped VJP) "
                  f"and a scatter of {sel.size} targets into {ns}; {dt:.1f}s",
    }


if __name__ == "__main__":
    main()
