#!/usr/bin/env python
"""Extremum-graph benchmark on one MI355X.

A step is one pass of the whole hot path (eg_build: classification,
pointer-jumping labels, saddle reps, arc sort / de-duplication, CSR) over one
field that is already resident in HBM.  Default workload: the 512^3 float32
Gaussian random field (seed 1, correlation length 8 voxels), maxima graph.

    python bench.py [--steps K] [--warmup W] [--workload grf512|2d256|5d32|6d16]

Prints one JSON line.  Besides the contract fields it carries
  roofline      the dominant kernel against the HBM peak (algorithmic bytes /
                its average duration, timed with HIP events on the launch stream)
  cpu_baseline  the CPU oracle timed on bounded slabs of the same field, on all
                host cores and on one (7 runs, best and worst dropped)
  stages_ms     per-stage times (classify / label / arcs), HIP events
  batched       256 fields of uneven sizes in one eg_build_batched per step,
                against one eg_build per field (default workload only)
  serving       the request loop on host-resident fields at 200 requests/s:
                p50/p99 latency (copy included), vertices/s, mean batch
                (default workload only)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "vertices/s + HBM GB/s for extremum graph (512³ f32); batched p99 latency"
VALU_PEAK_GINSTS = 256 * 4 * 2.4 / 4  # G wave64 VALU instructions/s (SIMD16: 4 cycles each)
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per vertex: classify reads f and writes the pointer;
# the whole path reads f, writes pointers, reads them and writes labels
CLASSIFY_BYTES_PER_VERTEX = 8
PATH_BYTES_PER_VERTEX = 16


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="grf512", choices=["grf512", "2d256", "5d32", "6d16", "batched", "serving"])
    ap.add_argument("--requests", type=int, default=2000, help="serving workload: number of requests")
    ap.add_argument("--rate", type=float, default=200.0, help="serving workload: Poisson arrival rate (1/s)")
    ap.add_argument("--sat-rate", type=float, default=50000.0,
                    help="serving workload: second arrival rate, above what one GPU sustains")
    ap.add_argument("--fields", type=int, default=256, help="batched workload: number of fields")
    ap.add_argument("--graph", action="store_true", help="batched workload: replay a captured HIP graph")
    ap.add_argument("--side", type=int, default=None, help="override the grid side (smoke runs)")
    ap.add_argument("--minima", action="store_true", help="minimum graph instead of maximum graph")
    ap.add_argument("--stage-reps", type=int, default=20, help="repetitions for the per-stage timings")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-paths", action="store_true", help="skip the gradient-path geometry measurement")
    ap.add_argument("--no-typed", action="store_true", help="skip the other-sample-type measurement")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched sub-measurement (256 fields)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving sub-measurement")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (library default tile shape and links per pass)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB three times (a reference for HBM byte counters)")
    ap.add_argument("--cpu-planes", type=int, default=None,
                    help="slab thickness (slowest axis) for the CPU oracle baseline")
    ap.add_argument("--profile-stage", default=None, choices=["classify", "label", "arcs"],
                    help="after the bench, run only this stage --stage-reps times (for counter runs)")
    return ap.parse_args()


# sources that define each profiled kernel (or the whole path): a counter
# summary stays valid only while these files are unchanged
KERNEL_SOURCES = {"k_classify": ("eg_classify_tiled.hip", "eg_internal.h", "eg_rows.h")}


def path_sources():
    d = os.path.join(ROOT, "paper_2303_02724_amd", "csrc")
    return tuple(sorted(n for n in os.listdir(d) if n.endswith((".hip", ".h", ".cpp"))))


def kernel_source_hash(kernel: str = "k_classify") -> str:
    d = os.path.join(ROOT, "paper_2303_02724_amd", "csrc")
    h = hashlib.sha256()
    for name in (path_sources() if kernel == "path" else KERNEL_SOURCES[kernel]):
        h.update(name.encode())
        with open(os.path.join(d, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_counter(prefix: str, key: str, kernel: str, workload: str, tile3):
    """A per-launch figure from a committed counter summary
    (profiles/<prefix>_<kernel>_<workload>.txt), used only if the summary was
    taken on the current kernel sources and the same tile shape (else None;
    tile3=None reads an unprefixed key)."""
    p = os.path.join(ROOT, "profiles", f"{prefix}_{kernel}_{workload}.txt")
    if not os.path.exists(p):
        return None
    vals = {}
    with open(p) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != kernel_source_hash(kernel):
        return None
    try:
        return float(vals[key if tile3 is None else f"tile3_{tile3}_{key}"])
    except (KeyError, ValueError):
        return None


def measure_paths(args, f, t, tuning):
    """Gradient-path geometry (eg_paths) of the same field, after a build with
    pointers: HIP-event time of the paths stage alone."""
    import torch

    from paper_2303_02724_amd import eg

    b = eg.Builder(f.shape, minima=args.minima, want_ptr=True, device=t.device, tuning=tuning)
    b.run(t)
    p = b.paths(t)  # sizes the path buffers
    npaths, nverts = int(p.path_offsets.numel()) - 1, int(p.vertices.numel())
    lengths = (p.path_offsets[1:] - p.path_offsets[:-1]).cpu()
    s = torch.cuda.current_stream()
    reps = max(3, args.stage_reps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.launch_paths(t, stream=s)
    e0.record(s)
    for _ in range(reps):
        b.launch_paths(t, stream=s)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    res = {"ms": round(ms, 4), "paths": npaths, "vertices": nverts,
           "longest": int(lengths.max()) if npaths else 0,
           "mean_length": round(float(lengths.float().mean()), 2) if npaths else 0.0,
           # per path vertex: its pointer and key read, its id written
           "GBs_at_12B_per_vertex": round(12 * nverts / (ms * 1e-3) / 1e9, 1)}
    del b, p
    torch.cuda.empty_cache()
    return res


def measure_typed(args, t, tuning):
    """Other sample types (eg_order_field, then the float32 path): the same
    field as float64 (the order surrogate sorts all 64 key bits), quantised to
    int32 (2^20 steps per unit) and to int16 (2^10 steps per unit).  HIP-event
    times of the surrogate alone and of surrogate plus build."""
    import torch

    from paper_2303_02724_amd import eg

    variants = {"f64": t.double(), "i32": torch.round(t.double() * 2.0 ** 20).to(torch.int32),
                "i16": torch.clamp(torch.round(t * 2.0 ** 10), -32768, 32767).to(torch.int16)}
    b = eg.Builder(t.shape, minima=args.minima, device=t.device, tuning=tuning)
    s = torch.cuda.current_stream()
    reps = max(3, args.stage_reps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    for name, x in variants.items():
        o = eg.Order(x.dtype, x.numel(), x.device)
        o.launch(x, s)
        e0.record(s)
        for _ in range(reps):
            o.launch(x, s)
        e1.record(s)
        e1.synchronize()
        order_ms = e0.elapsed_time(e1) / reps
        b.run(x)
        e0.record(s)
        for _ in range(reps):
            b.launch(x, stream=s)
        e1.record(s)
        e1.synchronize()
        total_ms = e0.elapsed_time(e1) / reps
        out[name] = {"order_ms": round(order_ms, 3), "build_ms": round(total_ms, 3),
                     "G_vertices_per_s": round(x.numel() / (total_ms * 1e-3) / 1e9, 2),
                     "order_workspace_MB": round(o.ws_bytes / 2 ** 20, 1)}
        del o
    del b, variants
    torch.cuda.empty_cache()
    return out


def measure_graph(b, t, steps):
    """The same build replayed from a captured HIP graph: the kernels are the
    same, only the host launch cost goes away (what matters for small fields).
    Replays are checked against the eager result."""
    import torch

    from paper_2303_02724_amd import eg

    ref = (b.maxima.clone(), b.arcs.clone(), b.labels.clone())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.launch(t, stream=side)  # warm the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        b.launch(t, stream=side)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    same = all(torch.equal(x, y) for x, y in zip(ref, (b.maxima, b.arcs, b.labels)))
    if not same or b.header_values()[eg.H_STATUS] != eg.EG_OK:
        return {"error": "graph replay differs from the eager build"}
    w0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - w0) / steps
    same = all(torch.equal(x, y) for x, y in zip(ref, (b.maxima, b.arcs, b.labels)))
    del g
    return {"ms_per_step": round(ms, 4), "vertices_per_s": t.numel() / (ms * 1e-3),
            "replays_equal_eager": bool(same)}


def measure_streamed(f, tuning, minima, reps=7, slab=32):
    """The field starting in pinned host memory (PCIe included): copied whole
    and then built (one stream), against eg_build_streamed (slabs of `slab`
    planes copied on a second stream while the slabs that have landed are
    classified).  Host wall time per build, 7 runs, best and worst dropped;
    the two results are compared."""
    import torch

    from paper_2303_02724_amd import eg

    host = torch.empty(f.shape, dtype=torch.float32, pin_memory=True)
    host.copy_(torch.from_numpy(f))
    b = eg.Builder(f.shape, minima=minima, tuning=tuning)
    b.run_streamed(host, slab)  # sizes the buffers
    dev = b.field_dev
    s = torch.cuda.current_stream()

    def whole():
        dev.copy_(host, non_blocking=True)
        b.launch(dev, stream=s)

    def streamed():
        b.launch_streamed(host, slab, stream=s)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts.sort()
        mid = ts[1:-1] if len(ts) > 2 else ts
        return sum(mid) / len(mid)

    t_whole = timed(whole)
    ref = (b.labels.clone(), b.arcs.clone(), b.header.clone())
    t_str = timed(streamed)
    same = all(torch.equal(x, y) for x, y in zip(ref, (b.labels, b.arcs, b.header)))
    N = int(f.size)
    out = {"slab_planes": slab, "slabs": -(-f.shape[0] // slab),
           "copy_then_build": {"ms": round(t_whole * 1e3, 3), "vertices_per_s": N / t_whole},
           "streamed": {"ms": round(t_str * 1e3, 3), "vertices_per_s": N / t_str},
           "speedup": t_whole / t_str, "results_equal": bool(same),
           "note": "PCIe-inclusive: the field starts in pinned host memory"}
    del b, host, dev
    torch.cuda.empty_cache()
    return out


def measure_simplify(res, t, minima, runs=3):
    """Graph simplification (host): arc bundling then persistence-directed
    cancellation at 5 % of the field's value range, as in the paper's
    experiments.  ms_host is eg_simplify on the host copy of the graph (median
    of `runs`); ms_gather the device gather of the critical values and the
    copy of the graph to the host, once."""
    import numpy as np
    import torch

    from paper_2303_02724_amd import eg

    thr = 0.05 * float(t.max() - t.min())
    flat = t.reshape(-1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    host = (res.maxima.cpu().numpy(), flat[res.maxima.long()].cpu().numpy().astype(np.float64),
            res.saddles.cpu().numpy(), flat[res.saddles.long()].cpu().numpy().astype(np.float64),
            res.arc_offsets.cpu().numpy(), res.arc_maxima.cpu().numpy())
    ms_gather = (time.perf_counter() - t0) * 1e3
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        s = eg.simplify_graph(*host, eg.SIMPLIFY_BUNDLE | eg.SIMPLIFY_CANCEL, thr, minima)
        ts.append((time.perf_counter() - t0) * 1e3)
    ms = sorted(ts)[len(ts) // 2]
    rows = s["arc_offsets"]
    return {"ms_host": round(ms, 3), "ms_gather": round(ms_gather, 3), "host_threads": os.cpu_count(),
            "threshold": thr, "cancellations": int(s["pair_saddle"].size),
            "maxima_left": int((s["max_rep"] == range(s["max_rep"].size)).sum()),
            "saddles_left": int((rows[1:] > rows[:-1]).sum()), "arcs_left": int(rows[-1]),
            "maxima_in": int(res.maxima.numel()), "saddles_in": int(res.saddles.numel()),
            "arcs_in": int(res.arc_maxima.numel())}


def make_field(args):
    from paper_2303_02724_amd import workloads as W

    if args.workload == "grf512":
        side = args.side or 512
        f = W.field_3d_grf(side, seed=1)
        cfg = {"workload": f"grf3d_{side}", "shape": [side] * 3, "seed": 1, "corr_len_voxels": 8,
               "field": "Gaussian random field, mean 0, std 1"}
    elif args.workload == "2d256":
        side = args.side or 256
        f = W.gaussian_mixture((side, side), 0, n_gauss=8, noise=1e-3)
        cfg = {"workload": f"gauss2d_{side}", "shape": [side] * 2, "seed": 0, "gaussians": 8, "noise": 1e-3}
    elif args.workload == "6d16":
        side = args.side or 16
        f = W.field_6d(side)
        cfg = {"workload": f"schwefel6d_{side}", "shape": [side] * 6,
               "field": "Schwefel function on [-500, 500]^6 (Table 4's 6D grids)"}
    else:
        side = args.side or 32
        f = W.field_5d_32(seed=2, side=side)
        cfg = {"workload": f"gauss5d_{side}", "shape": [side] * 5, "seed": 2, "gaussians": 16, "noise": 1e-4}
    cfg["mode"] = "minima" if args.minima else "maxima"
    return f, cfg


def time_stages(b, t, reps):
    """Average ms of each stage, HIP events on the launch stream."""
    import torch

    s = torch.cuda.current_stream()
    acc = {"classify": 0.0, "label": 0.0, "arcs": 0.0}
    for _ in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(s)
        b.launch(t, stream=s, stage="classify")
        ev[1].record(s)
        b.launch(t, stream=s, stage="label")
        ev[2].record(s)
        b.launch(t, stream=s, stage="arcs")
        ev[3].record(s)
        ev[3].synchronize()
        acc["classify"] += ev[0].elapsed_time(ev[1])
        acc["label"] += ev[1].elapsed_time(ev[2])
        acc["arcs"] += ev[2].elapsed_time(ev[3])
    return {k: v / reps for k, v in acc.items()}


def cpu_baseline(f, planes_all, planes_one, runs=7):
    """The oracle on slabs of the field (the first planes along the slowest
    axis), on all host cores and on one core: `runs` runs each, the best and
    the worst dropped, the mean of the rest (the paper's Sec. 5 protocol),
    with the median beside it."""
    from oracle import oracle as O

    def timed(sub):
        ts = []
        g = None
        for _ in range(runs):
            t0 = time.perf_counter()
            g = O.extremum_graph(sub)
            ts.append(time.perf_counter() - t0)
        ts.sort()
        trimmed = ts[1:-1] if len(ts) > 2 else ts
        return sum(trimmed) / len(trimmed), ts[len(ts) // 2], g

    cores = O.num_threads()
    sub = f[:planes_all]
    mean, med, g = timed(sub)
    prev = O.set_threads(1)
    try:
        sub1 = f[:planes_one]
        mean1, med1, _ = timed(sub1)
    finally:
        O.set_threads(prev)
    return {
        "value": sub.size / mean,
        "unit": "vertices/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"oracle (classification + labels + arcs) on the first {sub.shape[0]} of {f.shape[0]} "
                  f"slowest-axis planes, shape {list(sub.shape)}, {sub.size} vertices, {mean:.3f} s per run; "
                  f"{len(g['maxima'])} maxima, {len(g['saddles'])} saddles",
        "protocol": f"{runs} runs, best and worst dropped, mean of the rest",
        "median_value": sub.size / med,
        "one_core": {"value": sub1.size / mean1, "median_value": sub1.size / med1, "cores": 1,
                     "sample": f"first {sub1.shape[0]} planes, {sub1.size} vertices, {mean1:.3f} s per run"},
    }


def batched_fields(count):
    from paper_2303_02724_amd import workloads as W

    specs = W.batched_specs(count=count)
    return [W.batched_field(sp) for sp in specs]


def measure_batched(fields, steps, warmup, graph=True):
    """All fields in one eg_build_batched per step (the launch configuration
    picked on this batch), against the same fields built one eg_build at a
    time on the same stream; also the batch replayed from a captured HIP
    graph.  Host wall time over the steps, inputs resident."""
    import torch

    from paper_2303_02724_amd import eg

    dev = torch.device("cuda:0")
    ts = [torch.from_numpy(f).to(dev) for f in fields]
    N = sum(int(f.size) for f in fields)
    bb = eg.BatchBuilder([f.shape for f in fields], device=dev)
    bb.run(ts)  # sizes every field's buffers
    # exact-fit capacities keep the batch workspace small
    caps = []
    for b in bb.builders:
        h = b.header_values()
        caps.append({"cap_max": max(1, h[eg.H_NMAX]), "cap_sad": max(1, h[eg.H_NSAD]),
                     "cap_arc": max(1, h[eg.H_NARC])})
    s = torch.cuda.current_stream()

    def timed(step, n):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    # launch configuration for the batch: every 2D and 3D tile shape, timed
    # on this batch (identical results by construction)
    cands = {}
    for tu in (eg.tuning(0, 0), eg.tuning(2, 0), eg.tuning(1, 0), eg.tuning(0, 1), eg.tuning(2, 1)):
        cb = eg.BatchBuilder([f.shape for f in fields], device=dev, caps=caps, tuning=tu)
        cb.run(ts)
        cands[tu] = timed(lambda: cb.launch(stream=s), 3)
        del cb
    best = min(cands, key=cands.get)
    bb = eg.BatchBuilder([f.shape for f in fields], device=dev, caps=caps, tuning=best)
    bb.run(ts)
    tb = timed(lambda: bb.launch(stream=s), steps)
    heads = [b.header_values() for b in bb.builders]
    bad = [h for h in heads if h[eg.H_STATUS] != eg.EG_OK]
    if bad:
        raise SystemExit(f"device status after the batched steps: {bad[:3]}")
    tg = None
    if graph:
        side = torch.cuda.Stream()
        side.wait_stream(s)
        with torch.cuda.stream(side):
            bb.launch(stream=side)  # warm the capture stream
        s.wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            bb.launch(stream=side)
        torch.cuda.synchronize()
        tg = timed(g.replay, steps)
        del g
    for b, t in zip(bb.builders, ts):
        b.tuning = best
        b.out.tuning = best

    def per_field_step():
        for b, t in zip(bb.builders, ts):
            b.launch(t, stream=s)

    tp = timed(per_field_step, max(2, steps // 4))
    out = {"fields": len(fields), "vertices": N,
           "shapes": "2D sides U[64,2048] or 3D sides U[32,192], p = 1/2, meta-seed 3",
           "value": N / tb, "unit": "vertices/s", "ms_per_step": tb * 1e3,
           "tuning": {"choice": hex(best), "candidates_ms": {hex(k): round(v * 1e3, 3) for k, v in cands.items()}},
           "per_field": {"value": N / tp, "ms_per_step": tp * 1e3},
           "speedup_vs_per_field": tp / tb}
    if tg is not None:
        out["graph_replay"] = {"value": N / tg, "ms_per_step": tg * 1e3}
    del bb, ts
    torch.cuda.empty_cache()
    return out


def run_batched(args):
    """Batched workload: all fields in one eg_build_batched per step, against
    the same fields built one eg_build at a time on the same stream."""
    import torch

    t_gen = time.perf_counter()
    fields = batched_fields(args.fields)
    t_gen = time.perf_counter() - t_gen
    torch.cuda.set_device(torch.device("cuda:0"))
    m = measure_batched(fields, args.steps, args.warmup, graph=True)
    out = {
        "metric": METRIC,
        "value": m["value"],
        "unit": "vertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched_{len(fields)}", "fields": len(fields), "vertices": m["vertices"],
                   "shapes": m["shapes"]},
        "batched": m,
        "field_gen_s": round(t_gen, 2),
    }
    print(json.dumps(out), flush=True)


def serving_pool(n_requests, rate, seed=4, n_small=47, big_side=384, p_big=0.1):
    """Poisson arrivals; each request names one field: the big_side^3 field
    with probability p_big, else one of n_small fields whose shapes follow
    the batched workload (2D sides U[64,2048] or 3D sides U[32,192])."""
    from paper_2303_02724_amd import workloads as W

    specs = W.batched_specs(count=n_small, meta_seed=seed + 100)
    fields = [W.batched_field(sp) for sp in specs]
    fields.append(W.gaussian_mixture((big_side,) * 3, seed + 200, n_gauss=8, noise=1e-3))
    return fields, serving_requests(n_requests, rate, seed, n_small, p_big)


def serving_requests(n_requests, rate, seed=4, n_small=47, p_big=0.1):
    """(arrival_s, field index) pairs: Poisson arrivals at `rate`; index
    n_small (the big field) with probability p_big, else uniform."""
    import numpy as np

    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    reqs = []
    for _ in range(n_requests):
        t += rng.exponential(1.0 / rate)
        fi = n_small if rng.random() < p_big else int(rng.integers(0, n_small))
        reqs.append((t, fi))
    return reqs


def measure_serving(n_requests, rate, sat_rate):
    """The serving loop on host-resident (pinned) fields, copied to the device
    at admission: continuous batching against one request at a time, at the
    configured arrival rate and at one above what the GPU sustains.  Latency
    = completion seen by the host - arrival (copy included)."""
    import torch

    from paper_2303_02724_amd import eg, serving

    t_gen = time.perf_counter()
    host, reqs = serving_pool(n_requests, rate)
    t_gen = time.perf_counter() - t_gen
    dev = torch.device("cuda:0")
    fields = []
    caps = {}
    for f in host:
        p = torch.empty(f.shape, dtype=torch.float32, pin_memory=True)
        p.copy_(torch.from_numpy(f))
        fields.append(p)
        # capacities measured once per field shape (untimed), so no request retries
        r = eg.build(p.to(dev))
        caps[tuple(f.shape)] = {"cap_max": max(1, r.counts["maxima"]), "cap_sad": max(1, r.counts["saddles"]),
                                "cap_arc": max(1, r.counts["arcs"])}
    del r
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    policies = [("continuous_batching", dict(max_batch=32, lanes=3, max_slots=96)),
                ("one_at_a_time", dict(max_batch=1, lanes=1, max_slots=1))]
    servers = {}
    for name, kw in policies:
        srv = serving.Server(device=dev, caps_for=lambda sh: caps[sh], **kw)
        srv.prewarm([tuple(f.shape) for f in fields], per_shape=2 if kw["max_batch"] > 1 else 1)
        srv.run(reqs[: min(50, len(reqs))], fields)  # warm-up stream
        servers[name] = srv
    torch.cuda.synchronize()

    def measure(rq):
        res = {}
        for name, _ in policies:
            torch.cuda.synchronize()
            res[name] = servers[name].run(rq, fields).summary()
        return res

    out = measure(reqs)
    sat = measure(serving_requests(n_requests, sat_rate))
    cb, fifo = out["continuous_batching"], out["one_at_a_time"]
    res = {"rate_hz": rate, "requests": len(reqs),
           "fields": "host-resident (pinned), copied at admission: 47 batched-workload shapes + 384^3 with p = 0.1",
           "p50_ms": cb["p50_ms"], "p99_ms": cb["p99_ms"], "vertices_per_s": cb["vertices_per_s"],
           "mean_batch": cb["mean_batch"], "continuous_batching": cb, "one_at_a_time": fifo,
           "saturated": {"rate_hz": sat_rate, "continuous_batching": sat["continuous_batching"],
                         "one_at_a_time": sat["one_at_a_time"],
                         "throughput_ratio": sat["continuous_batching"]["vertices_per_s"] /
                         sat["one_at_a_time"]["vertices_per_s"]},
           "field_gen_s": round(t_gen, 2)}
    del servers, fields
    torch.cuda.empty_cache()
    return res


def run_serving(args):
    import torch

    torch.cuda.set_device(torch.device("cuda:0"))
    m = measure_serving(args.requests, args.rate, args.sat_rate)
    cb = m["continuous_batching"]
    res = {
        "metric": METRIC,
        "value": cb["vertices_per_s"],
        "unit": "vertices/s",
        "n_gpus": 1,
        "steps": m["requests"],
        "warmup": 50,
        "ms_per_step": cb["mean_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"serving_poisson_{int(args.rate)}hz", "requests": m["requests"],
                   "fields": m["fields"], "rate_hz": args.rate},
        "p50_ms": m["p50_ms"],
        "p99_ms": m["p99_ms"],
        "serving": m,
    }
    print(json.dumps(res), flush=True)


def main():
    args = parse()
    if args.workload == "batched" and args.gpus == 1:
        return run_batched(args)
    if args.workload == "serving" and args.gpus == 1:
        return run_serving(args)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2303_02724_amd import eg

    t_gen = time.perf_counter()
    f, cfg = make_field(args)
    t_gen = time.perf_counter() - t_gen
    N = int(f.size)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t = torch.from_numpy(f).to(dev)
    # H2D is reported apart from the timed region (inputs are resident when it starts)
    torch.cuda.synchronize()
    th = time.perf_counter()
    t2 = torch.from_numpy(f).to(dev)
    torch.cuda.synchronize()
    h2d_s = time.perf_counter() - th
    del t2

    if args.calibrate_copy:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings
        # convert the counters of the other kernels to HBM bytes
        n = args.calibrate_copy << 18  # float32 elements
        src = torch.ones(n, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
            torch.cuda.synchronize()
        del src, dst

    # the autotuner picks the launch configuration on this field (untimed);
    # every choice gives identical results
    tuning, tune_ms = 0, None
    if not args.no_tune:
        from paper_2303_02724_amd import tune

        tr = tune.tune(t, minima=args.minima, reps=5, path=None)
        tuning, tune_ms = tr["tuning"], tr["times_ms"]
        torch.cuda.empty_cache()

    b = eg.Builder(f.shape, minima=args.minima, device=dev, tuning=tuning)
    res = b.run(t)  # sizes the buffers (untimed)
    counts = dict(res.counts)
    counts["jump_passes"] = res.passes
    # saddles whose arcs reach at least two distinct maxima (the others have
    # beta >= 2 components that all end at one maximum)
    counts["separating_saddles"] = int((res.arc_offsets[1:] - res.arc_offsets[:-1] >= 2).sum().item())

    s = torch.cuda.current_stream()
    for _ in range(args.warmup):
        b.launch(t, stream=s)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(s)
    for _ in range(args.steps):
        b.launch(t, stream=s)
    ev1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_ms = ev0.elapsed_time(ev1)
    h = b.header_values()
    if h[eg.H_STATUS] != eg.EG_OK:
        raise SystemExit(f"device status {h[eg.H_STATUS]} after the timed region: {h}")
    ms_per_step = 1000.0 * wall / args.steps
    value = N * args.steps / wall

    stages = time_stages(b, t, args.stage_reps)
    dom = max(stages, key=stages.get)
    kernel_name = {"classify": "k_classify", "label": "k_exit_jump + k_final_tiled + k_final",
                   "arcs": "k_mask_* + k_arc_*"}[dom]
    # roofline of the classification kernel (one launch per step, 8 B/vertex)
    cls_ms = stages["classify"]
    alg_bytes = CLASSIFY_BYTES_PER_VERTEX * N
    achieved = alg_bytes / (cls_ms * 1e-3) / 1e9
    tile3 = tuning & 0xF
    traffic = recorded_counter("traffic", "traffic_bytes_per_launch", "k_classify", cfg["workload"], tile3)
    roof = {"bound": "hbm", "kernel": "k_classify (stages a + c)", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "algorithmic_bytes_per_launch": alg_bytes,
            "avg_launch_ms": round(cls_ms, 4), "dominant_stage": dom, "dominant_stage_kernel": kernel_name}
    # what actually limits the kernel: vector instruction issue (counted
    # wave64 instructions of one launch over its measured duration, against
    # 256 CUs x 4 SIMDs x 2.4 GHz with a wave64 instruction every 4 cycles)
    # the whole path: counted HBM bytes of one step (all kernels, default
    # launch configuration) over the live per-stage kernel time
    pbytes = recorded_counter("traffic", "path_traffic_bytes_per_step", "path", cfg["workload"], None)
    if pbytes is not None and (tuning & 0xF) == 0:
        path_ms = sum(stages.values())
        pg = pbytes / (path_ms * 1e-3) / 1e9
        roof["path_rocprof"] = {"traffic_bytes_per_step": pbytes, "kernel_ms_per_step": round(path_ms, 4),
                                "achieved": round(pg, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": round(pg / HBM_PEAK_GBS, 4),
                                "note": "(FETCH_SIZE + WRITE_SIZE) of every kernel of one step / the sum of the "
                                        "stage times; counts re-reads, unlike the 16 B/vertex effective_GBs"}
    valu = recorded_counter("valu", "sq_insts_valu_per_launch", "k_classify", cfg["workload"], tile3)
    if valu is not None:
        rate = valu / (cls_ms * 1e-3) / 1e9
        roof["valu_issue"] = {"insts_per_launch": valu, "achieved": round(rate, 1), "peak": VALU_PEAK_GINSTS,
                              "unit": "G wave64 instructions/s", "frac": round(rate / VALU_PEAK_GINSTS, 4)}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "vertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": cfg,
        "roofline": roof,
        "effective_GBs": round(PATH_BYTES_PER_VERTEX * N / (ms_per_step * 1e-3) / 1e9, 1),
        "gpu_event_ms_per_step": gpu_ms / args.steps,
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "counts": counts,
        "tuning": {"choice": hex(tuning), "candidates_ms": {hex(k): round(v, 4) for k, v in (tune_ms or {}).items()}},
        "h2d_ms": round(h2d_s * 1e3, 3),
        "field_gen_s": round(t_gen, 2),
    }
    out["graph_replay"] = measure_graph(b, t, args.steps)
    if not args.no_paths:
        out["paths"] = measure_paths(args, f, t, tuning)
    out["simplify"] = measure_simplify(res, t, args.minima)
    if f.ndim in (2, 3):
        out["streamed"] = measure_streamed(f, tuning, args.minima)
    if not args.no_typed:
        out["typed"] = measure_typed(args, t, tuning)
    if args.profile_stage:
        torch.cuda.synchronize()
        if args.profile_stage != "classify":
            b.launch(t, stream=s, stage="classify")
        if args.profile_stage == "arcs":
            b.launch(t, stream=s, stage="label")
        for _ in range(args.stage_reps):
            if args.profile_stage == "label":
                b.launch(t, stream=s, stage="classify")
            b.launch(t, stream=s, stage=args.profile_stage)
        torch.cuda.synchronize()
    del b
    torch.cuda.empty_cache()
    if args.workload == "grf512" and not args.no_batched:
        out["batched"] = measure_batched(batched_fields(args.fields), steps=10, warmup=2)
    if args.workload == "grf512" and not args.no_serving:
        out["serving"] = measure_serving(args.requests, args.rate, args.sat_rate)
    if not args.no_cpu_baseline:
        planes = args.cpu_planes
        if planes is None:
            planes = {"grf512": max(1, f.shape[0] // 8), "2d256": f.shape[0], "5d32": max(1, f.shape[0] // 8),
                      "6d16": max(1, f.shape[0] // 8)}[args.workload]
        one = {"grf512": max(1, f.shape[0] // 64), "2d256": f.shape[0], "5d32": max(1, f.shape[0] // 16),
               "6d16": max(1, f.shape[0] // 16)}[args.workload]
        out["cpu_baseline"] = cpu_baseline(f, planes, one)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
