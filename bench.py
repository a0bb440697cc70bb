"""CHERT hot-path benchmark on one MI355X.

Default workload (`--workload shots`): batched shots, 128 sources over four
per-node grids of uneven size (401x201, 801x401, 1201x301, 1701x351 at 10 m,
seeded synthetic structurally complex TTI+Q media, workloads.config4), qP
and qSV, forward-star radius 5.  One step = the whole hot path over that
batch: the surrogate-started per-node cache build of every grid
(chert_build_cache_surrogate: MLP warm start, Newton polish, plain fallback)
and one batched trace of tau_R, propagation predecessors and t* for all 256
(shot, mode) jobs (chert_trace_batch).  Inputs (per-node classes, the
trained surrogate) are resident in HBM before the timed region; the
surrogate is trained once before it.

Prints one JSON line.  `value` is shots/s over whole-step wall time; the
breakdown carries Hamiltonian solves/s (surrogate-started and plain, unique
bins), useful edge relaxations/s, the surrogate-vs-plain traveltime error
over every field, and per-kernel times.  `roofline` is the dominant
kernel's, measured with HIP events around its launches in the timed steps.
The CPU oracle is timed on a fixed subset of the step and extrapolated
(`cpu_baseline`).

Other workloads print their own line: `layered` (the 5-layer model, class
caches), `complex2d` (per-node caches of the 1701x351 model, k-means
ablation), `3d` (the 201x201x101 layered model), `ablation` (angular step
and star radius), `local` (the OEV-versus-MEV sweep on rock layer 1 with
slowness- and ray-sampled caches), `cells` (the cell network on the layered
model), `mspm` (CHERT against the MSPM baseline on the rock-table layers).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Hamiltonian solves/s; edge relaxations/s; shots/s, surrogate vs plain at 1e-4"
HBM_PEAK_GBS = 8000.0
LAUNCH_NAMES = ("per_round", "persistent", "frontier")
FP64_PEAK_TFLOPS = 78.6
FP64_VALU_PEAK_TOPS = 39.3  # 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz, one op per lane-cycle

# HBM traffic per dispatch of the relaxation kernels on this workload, from
# rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE runs of
# `bench.py --profile-steps 2` (see profiles/), scaled by what the same
# counters read for a 256 MiB device copy (FETCH_SIZE x2.0, WRITE_SIZE x1.0).
# Valid only for the kernel source it was measured on.
MEASURED_TRAFFIC = {
    "source": "paper_2609_26108_amd/csrc/trace.hip",
    "source_sha256_16": "7c4a616df9a01d8a",
    "fetch_scale": 2.0, "write_scale": 1.0,
    # workload -> kernel -> (FETCH_SIZE KiB, WRITE_SIZE KiB) per dispatch
    # (profiles/k_relax_tau__shots_4_grids_per_node.md: one step, 16 x 64
    # tiles, push group 4, 112 dispatches of each relaxation kernel)
    "kib_per_dispatch": {"shots": {"k_relax_tau": (861622.49, 10930.35),
                                   "k_relax_tree": (261086.43, 54668.11)}},
}


def measured_traffic_bytes(kernel, workload="layered"):
    """Calibrated HBM bytes per dispatch, or None if not measured for the
    current kernel source."""
    import hashlib
    path = os.path.join(ROOT, MEASURED_TRAFFIC["source"])
    h = hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]
    kib = MEASURED_TRAFFIC["kib_per_dispatch"].get(workload, {}).get(kernel)
    if kib is None or h != MEASURED_TRAFFIC["source_sha256_16"]:
        return None
    return 1024.0 * (kib[0] * MEASURED_TRAFFIC["fetch_scale"] + kib[1] * MEASURED_TRAFFIC["write_scale"])


# Executed FP64 work per dispatch of the surrogate-started build's kernels on
# the structurally complex workload (`bench.py --workload complex2d`), from
# rocprofv3 --pmc SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64
# SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_TRANS_F64 (see profiles/): wave
# instructions x 64 lanes, an FMA counted as two flops (lanes masked off by
# divergence count as executed).  Valid only for the sources it was measured
# on.
MEASURED_FP64 = {
    "sources": ["paper_2609_26108_amd/csrc/cache_build.hip",
                "paper_2609_26108_amd/csrc/physics.h", "paper_2609_26108_amd/csrc/mlp.h"],
    "sources_sha256_16": "7829c908b494a563",
    "flops_per_dispatch": {"k_warm_solve": 3.7921e11, "k_warm_window": 2.8714e11,
                           "k_warm_fold": 2.1870e10, "k_warm_predict": 5.3496e9},
}


def measured_fp64_flops(kernel):
    """Executed FP64 flops per dispatch, or None if not measured for the
    current sources."""
    import hashlib
    h = hashlib.sha256()
    for src in MEASURED_FP64["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest()[:16] != MEASURED_FP64["sources_sha256_16"]:
        return None
    return MEASURED_FP64["flops_per_dispatch"].get(kernel)


def useful_edges(nx, nz, ox, oz):
    """In-grid directed star edges = relaxations Dijkstra performs per field
    when every node is reachable."""
    return int(sum((nx - abs(a)) * (nz - abs(b)) for a, b in zip(ox, oz)))


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--profile-steps", type=int, default=0,
                   help="run only this many steps, no baseline (for rocprofv3)")
    p.add_argument("--tile", type=int, nargs=2, default=(0, 0), metavar=("TX", "TZ"),
                   help="relaxation tile shape (0 0 = library default)")
    p.add_argument("--push-group", type=int, default=0, help="offsets per push item (1, 2, 4)")
    p.add_argument("--launch", type=int, default=0,
                   help="relaxation launch: 0 tiles, one launch per round; 1 tiles, "
                        "persistent; 2 node frontier")
    p.add_argument("--autotune", action="store_true",
                   help="headline: let the autotuner pick tile, push group, launch and ordering")
    p.add_argument("--no-autotune", action="store_true",
                   help="complex2d, shots: trace with the default (or given) launch options")
    p.add_argument("--bucket", type=float, default=0.0,
                   help="node-frontier near/far bucket width (units of the smallest weight)")
    p.add_argument("--workload", choices=("shots", "layered", "complex2d", "3d", "ablation", "local", "cells",
                            "mspm", "blocks"),
                   default="shots",
                   help="shots: 128 shots over 4 uneven per-node grids, surrogate-started "
                        "caches + one batched trace per step (default, the headline line); "
                        "layered: the 5-layer model on class caches; "
                        "complex2d: per-node caches of the structurally complex model, "
                        "plain vs surrogate-started; 3d: the 3D layered model; ablation: "
                        "angular step and star radius against the finest setting; cells: "
                        "the cell network; mspm: CHERT against MSPM; blocks: the compact 3D "
                        "TTI model on the block network")
    p.add_argument("--plain-stride", type=int, default=64,
                   help="complex2d: time the plain per-node build on every n-th node")
    p.add_argument("--full-plain", action="store_true",
                   help="complex2d: also build the plain per-node cache for every node and "
                        "compare traveltimes at full size")
    p.add_argument("--train-media", type=int, default=1000,
                   help="complex2d: media in the surrogate's training cache (x 3 modes x 360)")
    p.add_argument("--train-steps", type=int, default=4000)
    p.add_argument("--cpu-nodes", type=int, default=40,
                   help="complex2d: nodes in the CPU oracle's cache-build sample")
    p.add_argument("--kmeans", type=int, nargs="*", default=[],
                   help="complex2d: also trace k-means class caches with these K")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only run 4 device-to-device copies of MIB MiB (HBM counter scale)")
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: there is no multi-GPU path "
              "(shots and cache entries would shard across GPUs with no communication).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2609_26108_amd as C
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        # a plain copy of known size: FETCH_SIZE/WRITE_SIZE per dispatch of
        # this kernel against its true byte count gives the counter scale
        n = args.copy_calibration * (1 << 20)
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "copies": 4}))
        return
    if args.workload == "complex2d":
        run_complex(args)
        return
    if args.workload == "shots":
        run_shots(args)
        return
    if args.workload == "3d":
        run_3d(args)
        return
    if args.workload == "ablation":
        run_ablation(args)
        return
    if args.workload == "local":
        run_local(args)
        return
    if args.workload == "cells":
        run_cells(args)
        return
    if args.workload == "mspm":
        run_mspm(args)
        return
    if args.workload == "blocks":
        run_blocks(args)
        return
    m = W.config2()
    K = len(m.layers)
    desc = C.cache_desc(n_dirs=m.n_dirs, modes=m.modes)
    classes = torch.from_numpy(np.stack(
        [C.chert_class_from_thomsen(*L.thomsen_args()).as_array() for L in m.layers])).to(dev)
    cid = torch.from_numpy(m.class_id.reshape(-1).astype(np.int32)).to(dev)
    lay = C.chert_cache_layout_of(desc, K)
    cache = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=dev)
    cws = torch.empty(max(C.chert_build_cache_workspace_bytes(desc, K), 1), dtype=torch.uint8,
                      device=dev)
    grid = C.make_grid(m.nx, m.nz, m.hx, m.hz, m.radius, cid)
    stats = C.TraceStats()
    opts = C.trace_opts(C.OUT_ALL, tile_x=args.tile[0], tile_z=args.tile[1], stats=stats,
                        push_group=args.push_group, launch=args.launch,
                        bucket_width=args.bucket)
    S = len(m.sources)
    n = m.n_nodes
    outs = {mode: dict(
        tau_r=torch.empty((S, n), dtype=torch.float64, device=dev),
        tau_i=torch.empty((S, n), dtype=torch.float64, device=dev),
        tstar=torch.empty((S, n), dtype=torch.float64, device=dev),
        pred_p=torch.empty((S, n), dtype=torch.int32, device=dev),
        pred_a=torch.empty((S, n), dtype=torch.int32, device=dev)) for mode in m.modes}
    batch = C.Batch()
    for mode in m.modes:
        batch.add(desc, cache, K, grid, mode, m.sources, **outs[mode])
    stream = torch.cuda.current_stream()
    tune = None
    if args.autotune:  # pick the launch options on this batch, outside the timed steps
        C.chert_build_cache(desc, classes, K, cache, cws, stream=stream)
        aws = torch.empty(C.chert_trace_autotune_workspace_bytes(batch, opts),
                          dtype=torch.uint8, device=dev)
        t0 = time.perf_counter()
        probe_ms = C.chert_trace_autotune(batch, opts, aws, stream=stream)
        tune = {"s": time.perf_counter() - t0, "probe_ms": probe_ms,
                "tile": [opts.tile_x, opts.tile_z], "push_group": opts.push_group,
                "launch": LAUNCH_NAMES[opts.launch], "bucket_width": opts.bucket_width}
        opts = C.trace_opts(C.OUT_ALL, tile_x=opts.tile_x, tile_z=opts.tile_z, stats=stats,
                            push_group=opts.push_group, launch=opts.launch,
                            bucket_width=opts.bucket_width)
        del aws
    tws = torch.empty(C.chert_trace_batch_workspace_bytes(batch, opts), dtype=torch.uint8,
                      device=dev)

    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for k in ("build", "trace")}
    acc = {"build": 0.0, "trace": 0.0}

    def step(timed=False):
        if timed:
            ev["build"][0].record(stream)
        C.chert_build_cache(desc, classes, K, cache, cws, stream=stream)
        if timed:
            ev["build"][1].record(stream)
            ev["trace"][0].record(stream)
        C.chert_trace_batch(batch, opts, tws, stream=stream)
        if timed:
            ev["trace"][1].record(stream)
            torch.cuda.synchronize()
            for k in acc:
                acc[k] += ev[k][0].elapsed_time(ev[k][1])

    if args.profile_steps:
        for _ in range(args.profile_steps):
            step()
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps}))
        return

    # warmup; its last step is profiled for every kernel to find the
    # dominant one
    for w in range(max(args.warmup, 1)):
        if w == max(args.warmup, 1) - 1:
            C.chert_prof_enable(True)
        step()
    torch.cuda.synchronize()
    prof_all = C.chert_prof_read()
    dom = max(prof_all, key=lambda k: prof_all[k][1])
    # timed region: HIP events bracket only the dominant kernel's launches
    C.chert_prof_enable(True, only=dom)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(timed=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = C.chert_prof_read()
    C.chert_prof_enable(False)
    ms = 1e3 * wall / args.steps

    # the same steps with the trace replayed as one HIP graph (per-round
    # launches, round budget from the eager runs): no host checks or table
    # uploads inside the step.  Reported beside the eager figure.
    graph_ms = None
    if args.launch == C.LAUNCH_PER_ROUND:
        budget = max(stats.rounds[0], stats.rounds[1]) + 4
        gopts = C.trace_opts(C.OUT_ALL, tile_x=opts.tile_x, tile_z=opts.tile_z,
                             push_group=opts.push_group, launch=C.LAUNCH_PER_ROUND,
                             bucket_width=opts.bucket_width, max_rounds=budget)
        gws = torch.empty(C.chert_trace_batch_workspace_bytes(batch, gopts), dtype=torch.uint8,
                          device=dev)
        gstream = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(gstream):
            graph = C.TraceGraph(batch, gopts, gws, stream=gstream)
            try:
                gst = C.TraceStats()
                for _ in range(2):  # warm-up replays
                    C.chert_build_cache(desc, classes, K, cache, cws, stream=gstream)
                    graph.launch(gstream)
                    graph.finish(gst, gstream)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    C.chert_build_cache(desc, classes, K, cache, cws, stream=gstream)
                    graph.launch(gstream)
                    graph.finish(gst, gstream)  # waits, checks convergence in the budget
                torch.cuda.synchronize()
                graph_ms = 1e3 * (time.perf_counter() - t0) / args.steps
            finally:
                graph.close()
        del gws

    ox, oz, L, b = C.chert_star_2d(m.radius, m.hx, m.hz, m.n_dirs)
    E = useful_edges(m.nx, m.nz, ox, oz)
    fields_per_step = 2 * len(m.modes)
    edges_per_step = E * fields_per_step
    solves_per_step = len(m.modes) * K * m.n_dirs
    build_ms = acc["build"] / args.steps
    trace_ms = acc["trace"] / args.steps

    # sanity: the last step's fields are finite at the far corner for qP
    tr = outs[m.modes[0]]["tau_r"][0, -1].item()
    if not np.isfinite(tr):
        raise RuntimeError("bench produced an unreachable far corner")

    kernels = {k: {"launches_per_step": v[0], "ms_per_step": v[1],
                   "avg_us": 1e3 * v[1] / max(v[0], 1)} for k, v in prof_all.items()}
    kernels[dom] = {"launches_per_step": prof[dom][0] / args.steps,
                    "ms_per_step": prof[dom][1] / args.steps,
                    "avg_us": 1e3 * prof[dom][1] / max(prof[dom][0], 1),
                    "timed_region": True}
    st = stats.as_dict()
    raw = st["edge_relaxations"]
    # Roofline of the dominant kernel.  The relaxation on a class cache keeps
    # tau tiles, class ids and the class-pair weight table on chip, so its
    # algorithmic work is FP64 VALU: one add and one compare per useful edge
    # relaxation; peak = 78.6 TFLOP/s (FMA counted twice) / 2 = 39.3 T ops/s.
    if dom in ("k_relax_tau", "k_relax_persist_tau", "k_front_relax"):
        per_launch_ops = 2.0 * edges_per_step / kernels[dom]["launches_per_step"]
        achieved = per_launch_ops / (kernels[dom]["avg_us"] * 1e-6) / 1e12
        traffic = measured_traffic_bytes(dom, "layered")
        roof = {"kernel": dom, "bound": "alu", "achieved": achieved,
                "peak": FP64_VALU_PEAK_TOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_VALU_PEAK_TOPS, "traffic": traffic,
                "work_per_launch": f"{per_launch_ops:.4g} FP64 ops (2 per useful edge)",
                "avg_launch_us": kernels[dom]["avg_us"],
                "hbm_gbs_measured": (traffic / (kernels[dom]["avg_us"] * 1e-6) / 1e9
                                     if traffic else None)}
    else:
        roof = {"kernel": dom, "bound": "alu", "achieved": None, "peak": 78.6,
                "unit": "TFLOP/s", "frac": None, "traffic": None}
    res = {
        "metric": METRIC,
        "value": edges_per_step / (wall / args.steps),
        "unit": "useful edge relaxations/s (whole step: cache build + 6 fields)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded workloads.config2)",
        "config": {"workload": "5-layer TTI 401x201 @5 m, 5 classes, qP/qSV/qSH, "
                               "360-direction cache, radius 5, 1 surface source",
                   "nx": m.nx, "nz": m.nz, "classes": K, "modes": list(m.modes),
                   "radius": m.radius, "n_dirs": m.n_dirs, "sources": S,
                   "parallelism": "single GPU"},
        "breakdown": {
            "build_ms": build_ms, "trace_ms": trace_ms,
            "hamiltonian_solves_per_s": solves_per_step / (build_ms * 1e-3),
            "edge_relaxations_per_s_trace_only": edges_per_step / (trace_ms * 1e-3),
            "shots_per_s": len(m.modes) * S / (wall / args.steps),
            "useful_edges_per_field": E, "solves_per_step": solves_per_step,
            "trace_stats_last_step": st,
            "raw_over_useful": {"tau": raw[0] / edges_per_step, "tree": raw[1] / edges_per_step},
            "graph_ms_per_step": graph_ms,
            "launch": {"tile": [opts.tile_x or 32, opts.tile_z or 32],
                       "push_group": opts.push_group or 2, "launch": LAUNCH_NAMES[opts.launch],
                       "bucket_width": opts.bucket_width, "autotune": tune},
            "kernels": kernels,
        },
        "roofline": roof,
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(m, E, fields_per_step)
    print(json.dumps(res))


def cpu_baseline(m, E, fields_per_step):
    """The CPU oracle, as it stands, on one full step of the same workload."""
    import oracle as O
    O.build(force=False)
    cls = np.stack([O.class_from_thomsen(*L.thomsen_args()) for L in m.layers])
    mask = sum(1 << mo for mo in m.modes)
    t0 = time.perf_counter()
    f, s = O.build_cache_2d(cls, n_dirs=m.n_dirs, mode_mask=mask)
    t1 = time.perf_counter()
    for mode in m.modes:
        O.trace_2d(m.nx, m.nz, m.hx, m.hz, m.class_id, m.radius, f[0, mode], f[1, mode],
                   s[mode], m.sources[0])
    t2 = time.perf_counter()

    # the same step with one host thread per mode (each runs the serial
    # oracle: its cache build for that mode, then its Dijkstra runs)
    from concurrent.futures import ThreadPoolExecutor

    def one_mode(mode):
        fm, sm = O.build_cache_2d(cls, n_dirs=m.n_dirs, mode_mask=1 << mode)
        O.trace_2d(m.nx, m.nz, m.hx, m.hz, m.class_id, m.radius, fm[0, mode], fm[1, mode],
                   sm[mode], m.sources[0])

    t3 = time.perf_counter()
    with ThreadPoolExecutor(len(m.modes)) as ex:
        list(ex.map(one_mode, m.modes))
    t4 = time.perf_counter()
    return {"value": E * fields_per_step / (t2 - t0),
            "unit": "useful edge relaxations/s (whole step: cache build + 6 fields)",
            "cores": 1, "kind": "oracle",
            "sample": "one full step of the same workload (cache build + Dijkstra for 3 modes)",
            "build_s": t1 - t0, "trace_s": t2 - t1, "cpu_count": os.cpu_count(),
            "threads_per_mode": {"value": E * fields_per_step / (t4 - t3),
                                 "cores": len(m.modes), "s": t4 - t3,
                                 "sample": "the same step, one thread per mode (the oracle "
                                           "is serial within a mode)"}}


# --------------------------------------------------------------------------
# Per-node caches of the structurally complex model (1701 x 351 at 10 m,
# qSV, radius 5): plain vs surrogate-started cache build, traveltimes, and
# optionally coarse k-means class caches against the per-node fields.

def _events(torch, stream):
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    return a, b


def _elapsed(torch, ev, stream):
    ev[1].record(stream)
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[1]) * 1e-3


def _batch_relax_profile(C, torch, call, kernel):
    """One more call of a batched trace with the library's per-kernel timers
    on for `kernel` and statistics: (kernel seconds, pair relaxations,
    launches)."""
    st = C.TraceStats()
    C.chert_prof_enable(True, only=kernel)
    call(st)
    torch.cuda.synchronize()
    prof = C.chert_prof_read()
    C.chert_prof_enable(False)
    n, ms = prof.get(kernel, (0, 0.0))
    return ms * 1e-3, st.edge_relaxations[0], n


def _converged(status):
    ok = (status & (1 | 4 | 8)) == 0  # not NO_BRACKET / FLUID / NONPHYS
    return int(ok.sum())


def _tau_rel(a, b):
    fin = np.isfinite(b)
    same = bool(np.array_equal(np.isfinite(a), fin))
    rel = np.abs(a[fin] - b[fin]) / np.maximum(np.abs(b[fin]), 1e-300)
    return {"max": float(rel.max()), "median": float(np.median(rel)),
            "p99": float(np.quantile(rel, 0.99)), "same_reachability": same}


def train_surrogate(args, dev, stream):
    """Train the cache-solve surrogate on plain-solver entries of seeded
    media (full direction set, 3 modes); returns (blob, info)."""
    import torch
    import paper_2609_26108_amd as C
    import workloads as W
    t_rows = W.surrogate_training_rows(args.train_media)
    Kt = t_rows.shape[0]
    t_cls = torch.empty((Kt, 13), dtype=torch.float64, device=dev)
    C.chert_classes_from_thomsen(torch.from_numpy(t_rows).to(dev), t_cls)
    t_desc = C.cache_desc(modes=(0, 1, 2))
    t_lay = C.chert_cache_layout_of(t_desc, Kt)
    t_cache = torch.zeros(t_lay.total_bytes, dtype=torch.uint8, device=dev)
    ev = _events(torch, stream)
    C.chert_build_cache(t_desc, t_cls, Kt, t_cache, None, stream=stream)
    t_build = _elapsed(torch, ev, stream)
    ns = 3 * Kt * 360
    x = torch.empty((ns, 16), dtype=torch.float32, device=dev)
    y = torch.empty((ns, 4), dtype=torch.float32, device=dev)
    ok = torch.empty(ns, dtype=torch.int32, device=dev)
    C.chert_surrogate_dataset(t_desc, t_cache, t_cls, Kt, x, y, ok, stream=stream)
    lay = C.chert_surrogate_layout_of()
    blob = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=dev)
    C.chert_surrogate_init(blob, torch.from_numpy(W.mlp_init(C.SURROGATE_SHAPES, seed=1)).to(dev),
                           stream=stream)
    C.chert_surrogate_fit_norm(blob, x, y, ok, stream=stream)
    C.chert_prof_enable(True, only="k_sg_grad")
    ev = _events(torch, stream)
    losses = C.train_surrogate(blob, x, y, ok, steps=args.train_steps, batch=2048, seed=2,
                               stream=stream)
    t_train = _elapsed(torch, ev, stream)
    pg = C.chert_prof_read()["k_sg_grad"]
    C.chert_prof_enable(False)
    L = losses.cpu().numpy()
    # forward 2*(16*128 + 2*128*128 + 128*4) FLOP per sample, backward twice that
    flop_step = 3 * 2 * (16 * 128 + 2 * 128 * 128 + 128 * 4) * 2048
    grad_us = 1e3 * pg[1] / max(pg[0], 1)
    info = {
        "media": Kt, "samples_usable": int(ok.sum().item()), "steps": args.train_steps,
        "batch": 2048, "build_training_cache_s": t_build, "train_s": t_train,
        "loss_first20": float(L[:20].mean()), "loss_last200": float(L[-200:].mean()),
        "k_sg_grad_avg_us": grad_us,
        "k_sg_grad_mfma_frac": flop_step / (grad_us * 1e-6) / 2.5e15}

    return blob, info


def run_complex(args):
    import torch
    import paper_2609_26108_amd as C
    import workloads as W
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    m = W.complex_2d()
    rows = m.param_rows()
    n = rows.shape[0]
    params = torch.from_numpy(rows).to(dev)
    classes = torch.empty((n, 13), dtype=torch.float64, device=dev)
    C.chert_classes_from_thomsen(params, classes)
    mode = m.modes[0]
    sub = C.star_subset(m.radius, m.hx, m.hz)
    desc = C.cache_desc(modes=(mode,), subset=sub)
    out = {"metric": METRIC, "workload": "complex2d", "n_gpus": 1, "dtype": "f64",
           "data": "synthetic (seeded workloads.complex_2d)",
           "config": {"workload": f"structurally complex 2D, {m.nx}x{m.nz} @10 m, per-node "
                                  "TTI+Q, qSV, radius 5, star-bin subset cache",
                      "nodes": n, "columns": int(desc.n_cols), "sources": m.sources}}

    blob, out["training"] = train_surrogate(args, dev, stream)

    # 2. surrogate-started per-node build of every node
    lay_c = C.chert_cache_layout_of(desc, n)
    warm = torch.zeros(lay_c.total_bytes, dtype=torch.uint8, device=dev)
    wws = torch.empty(C.chert_build_cache_surrogate_workspace_bytes(desc, n), dtype=torch.uint8,
                      device=dev)
    wst = torch.zeros(C.WARM_NSTATS, dtype=torch.int64, device=dev)
    C.chert_build_cache_surrogate(desc, classes, n, blob, warm, wws, wst, stream=stream)  # warm-up
    torch.cuda.synchronize()
    C.chert_prof_enable(True)
    ev = _events(torch, stream)
    C.chert_build_cache_surrogate(desc, classes, n, blob, warm, wws, wst, stream=stream)
    t_warm = _elapsed(torch, ev, stream)
    pw = C.chert_prof_read()
    C.chert_prof_enable(False)
    fw, sw = C.cache_views(warm, desc, n)
    conv_warm = _converged(sw[mode].cpu().numpy())
    wstats = dict(zip(C.WARM_STATS, wst.cpu().numpy().tolist()))
    out["warm"] = {"build_s": t_warm, "converged_entries": conv_warm,
                   "hamiltonian_solves_per_s": conv_warm / t_warm, "stats": wstats,
                   "fallback_job_frac": wstats["fallback_jobs"] / max(wstats["jobs"], 1),
                   "kernels_ms": {k: v[1] for k, v in pw.items()}}
    # roofline of the build's dominant kernel: FP64 VALU work (executed
    # flops from the committed counter profile) over its live launch time
    dom = max(pw, key=lambda k: pw[k][1])
    fl = measured_fp64_flops(dom)
    avg_s = 1e-3 * pw[dom][1] / max(pw[dom][0], 1)
    ach = fl / avg_s / 1e12 if fl else None
    out["roofline"] = {
        "kernel": dom, "bound": "fp64", "achieved": ach, "peak": FP64_PEAK_TFLOPS,
        "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS if ach else None, "traffic": None,
        "avg_launch_us": 1e6 * avg_s,
        "work_per_launch": (f"{fl:.4g} executed FP64 flops (counters, 64 lanes per wave "
                            "instruction, FMA = 2)") if fl else None,
        "build_fp64_tflops": None}
    if fl:  # the whole build: every profiled kernel's FP64 work over its wall time
        flops = sum((measured_fp64_flops(k) or 0.0) * pw[k][0] for k in pw)
        out["roofline"]["build_fp64_tflops"] = flops / t_warm / 1e12

    # 3. plain per-node build on every plain_stride-th node (timing sample)
    pick = np.arange(0, n, args.plain_stride)
    cls_s = classes[torch.from_numpy(pick).to(dev)].contiguous()
    ks = pick.size
    lay_s = C.chert_cache_layout_of(desc, ks)
    plain_s = torch.zeros(lay_s.total_bytes, dtype=torch.uint8, device=dev)
    ev = _events(torch, stream)
    C.chert_build_cache(desc, cls_s, ks, plain_s, None, stream=stream)
    t_plain_s = _elapsed(torch, ev, stream)
    fp_s, sp_s = C.cache_views(plain_s, desc, ks)
    conv_s = _converged(sp_s[mode].cpu().numpy())
    fwn = fw[:, mode].cpu().numpy()[:, pick]
    fpn = fp_s[:, mode].cpu().numpy()
    okm = (sp_s[mode].cpu().numpy() & (1 | 4 | 8)) == 0
    same_status = bool(np.array_equal(sw[mode].cpu().numpy()[pick], sp_s[mode].cpu().numpy()))
    relV = np.abs(fwn[0][okm] - fpn[0][okm]) / fpn[0][okm]
    out["plain_sample"] = {"nodes": int(ks), "stride": args.plain_stride, "build_s": t_plain_s,
                           "converged_entries": conv_s,
                           "hamiltonian_solves_per_s": conv_s / t_plain_s,
                           "warm_vs_plain_same_status": same_status,
                           "warm_vs_plain_V_rel_max": float(relV.max()) if relV.size else 0.0}
    out["surrogate_speedup_solves_per_s"] = (conv_warm / t_warm) / (conv_s / t_plain_s)

    # 4. per-node traveltimes through the surrogate-started cache
    grid = C.make_grid(m.nx, m.nz, m.hx, m.hz, m.radius, None)
    stats = C.TraceStats()
    outs = C.OUT_TAU_R | C.OUT_TAU_I | C.OUT_TSTAR | C.OUT_PRED_P
    opts = C.trace_opts(outs, stats=stats, launch=args.launch, bucket_width=args.bucket)
    S = len(m.sources)
    tr = {k: torch.empty((S, n), dtype=torch.float64, device=dev) for k in ("r", "i", "t")}
    pp = torch.empty((S, n), dtype=torch.int32, device=dev)
    # launch options for this trace, picked by the autotuner before it is timed
    if not args.no_autotune:
        tb = C.Batch()
        tb.add(desc, warm, n, grid, mode, m.sources, tau_r=tr["r"], tau_i=tr["i"],
               tstar=tr["t"], pred_p=pp)
        aws = torch.empty(C.chert_trace_autotune_workspace_bytes(tb, opts), dtype=torch.uint8,
                          device=dev)
        C.chert_trace_autotune(tb, opts, aws, stream=stream)
        out["trace_autotune"] = {"tile": [opts.tile_x, opts.tile_z],
                                 "push_group": opts.push_group,
                                 "launch": LAUNCH_NAMES[opts.launch],
                                 "bucket_width": opts.bucket_width}
        opts = C.trace_opts(outs, opts.tile_x, opts.tile_z, push_group=opts.push_group,
                            launch=opts.launch, bucket_width=opts.bucket_width, stats=stats)
        del aws, tb
    tws = torch.empty(C.chert_trace_workspace_bytes(desc, n, grid, S, opts), dtype=torch.uint8,
                      device=dev)

    def trace(cache):
        ev = _events(torch, stream)
        C.chert_trace_field(desc, cache, n, grid, mode, m.sources, opts, tr["r"], tr["i"],
                            tr["t"], pp, None, tws, stream=stream)
        return _elapsed(torch, ev, stream)
    trace(warm)
    t_trace = trace(warm)
    tau_warm = tr["r"][0].cpu().numpy().copy()
    ox, oz, _, _ = C.chert_star_2d(m.radius, m.hx, m.hz, 360)
    E = useful_edges(m.nx, m.nz, ox, oz)
    out["trace"] = {"fields": "tau_R, tau_I, pred_P, t*", "trace_s": t_trace,
                    "useful_edges_per_field": E, "stats": stats.as_dict(),
                    "edge_relaxations_per_s_tau_fields": 2 * E / t_trace}
    if args.full_plain:
        plain = torch.zeros(lay_c.total_bytes, dtype=torch.uint8, device=dev)
        ev = _events(torch, stream)
        C.chert_build_cache(desc, classes, n, plain, None, stream=stream)
        t_plain = _elapsed(torch, ev, stream)
        trace(plain)
        out["plain_full"] = {"build_s": t_plain,
                             "converged_entries": _converged(C.cache_views(plain, desc, n)[1][mode].cpu().numpy()),
                             "tau_R_rel_warm_vs_plain": _tau_rel(tau_warm, tr["r"][0].cpu().numpy())}
        out["plain_full"]["hamiltonian_solves_per_s"] = out["plain_full"]["converged_entries"] / t_plain
        del plain

    # 5. coarse k-means class caches against the per-node field
    if args.kmeans:
        out["kmeans"] = {}
        for K in args.kmeans:
            crow, cid = W.kmeans_classes(m, K, seed=W.seed_for(3))
            kc = torch.empty((crow.shape[0], 13), dtype=torch.float64, device=dev)
            C.chert_classes_from_thomsen(torch.from_numpy(crow).to(dev), kc)
            kd = C.cache_desc(modes=(mode,))
            klay = C.chert_cache_layout_of(kd, crow.shape[0])
            kcache = torch.zeros(klay.total_bytes, dtype=torch.uint8, device=dev)
            C.chert_build_cache(kd, kc, crow.shape[0], kcache, torch.empty(
                max(C.chert_build_cache_workspace_bytes(kd, crow.shape[0]), 1), dtype=torch.uint8,
                device=dev), stream=stream)
            kg = C.make_grid(m.nx, m.nz, m.hx, m.hz, m.radius,
                             torch.from_numpy(cid.reshape(-1).astype(np.int32)).to(dev))
            ko = C.trace_opts(C.OUT_TAU_R)
            kt = torch.empty((S, n), dtype=torch.float64, device=dev)
            kws = torch.empty(C.chert_trace_workspace_bytes(kd, crow.shape[0], kg, S, ko),
                              dtype=torch.uint8, device=dev)
            ev = _events(torch, stream)
            C.chert_trace_field(kd, kcache, crow.shape[0], kg, mode, m.sources, ko, kt, None,
                                None, None, None, kws, stream=stream)
            t_k = _elapsed(torch, ev, stream)
            out["kmeans"][str(K)] = {"classes_incl_water": int(crow.shape[0]), "trace_s": t_k,
                                     "tau_R_rel_vs_per_node": _tau_rel(kt[0].cpu().numpy(), tau_warm)}
    if not args.no_cpu:
        solid = pick[rows[pick, 1] > 0.0][:args.cpu_nodes]
        out["cpu_baseline"] = cpu_baseline_complex(m, rows, sub, solid)
    out["value"] = out["warm"]["hamiltonian_solves_per_s"]
    out["unit"] = "converged per-node cache entries/s (surrogate-started build)"
    out["higher_is_better"] = True
    print(json.dumps(out))




def shot_models():
    """The batched-shots workload (workloads.config4)."""
    import workloads as W
    return W.config4()


def run_shots(args):
    """The batched-shots workload (the default line): 128 sources over four
    uneven per-node grids, qP and qSV.  One step = the surrogate-started
    per-node cache build of every grid (both modes) and one eager batched
    trace of tau_R, propagation predecessors and t* for all 256 (shot, mode)
    jobs.  The surrogate is trained once before the steps; the plain
    per-node build is timed beside them, and the traveltimes through the
    surrogate-started caches are compared with those through the plain
    caches over every field."""
    import torch
    import paper_2609_26108_amd as C
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    models = shot_models()
    outs_mask = C.OUT_TAU_R | C.OUT_PRED_P | C.OUT_TSTAR
    profiling = args.profile_steps > 0
    blob, tinfo = train_surrogate(args, dev, stream)
    ox, oz, _, _ = C.chert_star_2d(5, 10.0, 10.0, 360)
    n_off = len(ox)
    grids = []
    b_warm, b_plain = C.Batch(), C.Batch()
    for m in models:
        rows = m.param_rows()
        n = rows.shape[0]
        cls = torch.empty((n, 13), dtype=torch.float64, device=dev)
        C.chert_classes_from_thomsen(torch.from_numpy(rows).to(dev), cls)
        sub = C.star_subset(5, m.hx, m.hz)
        desc = C.cache_desc(modes=(0, 1), subset=sub)
        lay = C.chert_cache_layout_of(desc, n)
        warm = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=dev)
        plain = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=dev)
        wws = torch.empty(C.chert_build_cache_surrogate_workspace_bytes(desc, n),
                          dtype=torch.uint8, device=dev)
        wst = torch.zeros(C.WARM_NSTATS, dtype=torch.int64, device=dev)
        grid = C.make_grid(m.nx, m.nz, m.hx, m.hz, m.radius, None)
        S = len(m.sources)
        outs = {}
        for mode in (0, 1):
            out = dict(tau_r=torch.empty((S, n), dtype=torch.float64, device=dev),
                       tstar=torch.empty((S, n), dtype=torch.float64, device=dev),
                       pred_p=torch.empty((S, n), dtype=torch.int32, device=dev))
            b_warm.add(desc, warm, n, grid, mode, m.sources, **out)
            b_plain.add(desc, plain, n, grid, mode, m.sources, **out)
            outs[mode] = out
        grids.append(dict(m=m, n=n, cls=cls, desc=desc, sub=sub, warm=warm, plain=plain,
                          wws=wws, wst=wst, grid=grid, outs=outs))
    shots = 2 * sum(len(m.sources) for m in models)

    def build_warm():
        for g in grids:
            C.chert_build_cache_surrogate(g["desc"], g["cls"], g["n"], blob, g["warm"], g["wws"],
                                          g["wst"], stream=stream)

    # launch options of the trace: the autotuner's pick on this batch, or
    # the ones given on the command line
    build_warm()
    tune = None
    opts = C.trace_opts(outs_mask, tile_x=args.tile[0], tile_z=args.tile[1],
                        push_group=args.push_group, launch=args.launch, bucket_width=args.bucket)
    if not args.no_autotune and not profiling and args.tile == (0, 0):
        aws = torch.empty(C.chert_trace_autotune_workspace_bytes(b_warm, opts), dtype=torch.uint8,
                          device=dev)
        t0 = time.perf_counter()
        probe_ms = C.chert_trace_autotune(b_warm, opts, aws, stream=stream)
        tune = {"s": time.perf_counter() - t0, "probe_ms": probe_ms}
        del aws
    stats = C.TraceStats()
    opts = C.trace_opts(outs_mask, opts.tile_x, opts.tile_z, push_group=opts.push_group,
                        launch=opts.launch, bucket_width=opts.bucket_width, stats=stats)
    tws = torch.empty(C.chert_trace_batch_workspace_bytes(b_warm, opts), dtype=torch.uint8,
                      device=dev)
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for k in ("build", "trace")}
    acc = {"build": 0.0, "trace": 0.0}

    def step(timed=False):
        if timed:
            ev["build"][0].record(stream)
        build_warm()
        if timed:
            ev["build"][1].record(stream)
            ev["trace"][0].record(stream)
        C.chert_trace_batch(b_warm, opts, tws, stream=stream)
        if timed:
            ev["trace"][1].record(stream)
            torch.cuda.synchronize()
            for k in acc:
                acc[k] += ev[k][0].elapsed_time(ev[k][1])

    if profiling:
        for _ in range(args.profile_steps):
            step()
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps, "workload": "shots",
                          "tile": [opts.tile_x, opts.tile_z], "push_group": opts.push_group}))
        return

    # warm-up steps; the last one is profiled for every kernel (HIP events
    # around each launch) to find the dominant kernel
    for w in range(max(args.warmup, 1)):
        if w == max(args.warmup, 1) - 1:
            C.chert_prof_enable(True)
        step()
    torch.cuda.synchronize()
    prof_all = C.chert_prof_read()
    dom = max(prof_all, key=lambda k: prof_all[k][1])
    # timed region: HIP events bracket only the dominant kernel's launches
    C.chert_prof_enable(True, only=dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(timed=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = C.chert_prof_read()
    C.chert_prof_enable(False)
    ms = 1e3 * wall / args.steps
    build_ms = acc["build"] / args.steps
    trace_ms = acc["trace"] / args.steps

    # counters of the last step: unique solves (centrosymmetric copies are
    # not solves), useful edges over reachable nodes
    solves = 0
    wstats = {k: 0 for k in C.WARM_STATS}
    for g in grids:
        st = C.cache_views(g["warm"], g["desc"], g["n"])[1][:2].cpu().numpy()
        solves += _converged(st) // 2
        for k, v in zip(C.WARM_STATS, g["wst"].cpu().numpy().tolist()):
            wstats[k] += v
    useful = 0
    for g in grids:
        m = g["m"]
        # in-grid star edges out of each node
        ix = np.arange(m.nx)[None, :]
        iz = np.arange(m.nz)[:, None]
        cnt = np.zeros((m.nz, m.nx), np.int64)
        for a, c in zip(ox, oz):
            cnt += ((ix + a >= 0) & (ix + a < m.nx) & (iz + c >= 0) & (iz + c < m.nz))
        cnt_d = torch.from_numpy(cnt.reshape(-1)).to(dev)
        for mode in (0, 1):
            reach = torch.isfinite(g["outs"][mode]["tau_r"]).to(torch.int64)
            useful += int((reach * cnt_d[None, :]).sum().item())

    # the whole batch as one graph replay (per-round launches with a round
    # budget from the eager run), beside the eager figure
    graph_s = None
    if opts.launch == C.LAUNCH_PER_ROUND:
        gopts = C.trace_opts(outs_mask, opts.tile_x, opts.tile_z, push_group=opts.push_group,
                             launch=C.LAUNCH_PER_ROUND, bucket_width=opts.bucket_width,
                             max_rounds=max(stats.rounds) + 16)
        gs = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(gs):
            graph = C.TraceGraph(b_warm, gopts, tws, stream=gs)
            try:
                graph.launch(gs)
                graph.finish(None, gs)
                e0 = _events(torch, gs)
                reps = 3
                for _ in range(reps):
                    graph.launch(gs)
                graph.finish(None, gs)
                graph_s = _elapsed(torch, e0, gs) / reps
            finally:
                graph.close()

    # the persistent form of the same batch (one launch per phase with the
    # device-wide barrier between rounds) as a graph replay, for comparison
    pgraph_s = None
    if opts.launch in (C.LAUNCH_PER_ROUND, C.LAUNCH_PERSISTENT):
        popts = C.trace_opts(outs_mask, opts.tile_x, opts.tile_z, push_group=opts.push_group,
                             launch=C.LAUNCH_PERSISTENT, bucket_width=opts.bucket_width)
        if C.chert_trace_batch_workspace_bytes(b_warm, popts) <= tws.numel():
            gs = torch.cuda.Stream()
            torch.cuda.synchronize()
            with torch.cuda.stream(gs):
                graph = C.TraceGraph(b_warm, popts, tws, stream=gs)
                try:
                    graph.launch(gs)
                    graph.finish(None, gs)
                    e0 = _events(torch, gs)
                    reps = 3
                    for _ in range(reps):
                        graph.launch(gs)
                    graph.finish(None, gs)
                    pgraph_s = _elapsed(torch, e0, gs) / reps
                finally:
                    graph.close()

    # plain per-node build of every grid (timed once, after one warm-up grid)
    C.chert_build_cache(grids[0]["desc"], grids[0]["cls"], grids[0]["n"], grids[0]["plain"],
                        None, stream=stream)
    e0 = _events(torch, stream)
    for g in grids:
        C.chert_build_cache(g["desc"], g["cls"], g["n"], g["plain"], None, stream=stream)
    plain_s = _elapsed(torch, e0, stream)
    same_status = all(torch.equal(C.cache_views(g["warm"], g["desc"], g["n"])[1][:2],
                                  C.cache_views(g["plain"], g["desc"], g["n"])[1][:2])
                      for g in grids)

    # surrogate form vs plain form over every field: the same batch traced
    # through the plain caches
    warm_tau = [g["outs"][mode]["tau_r"].clone() for g in grids for mode in (0, 1)]
    C.chert_trace_batch(b_plain, opts, tws, stream=stream)
    torch.cuda.synchronize()
    worst, same_reach = 0.0, True
    for a, b in zip(warm_tau, [g["outs"][mode]["tau_r"] for g in grids for mode in (0, 1)]):
        fin = torch.isfinite(b)
        same_reach &= bool(torch.equal(torch.isfinite(a), fin))
        rel = (a[fin] - b[fin]).abs() / b[fin].abs().clamp_min(1e-300)
        worst = max(worst, float(rel.max().item()) if rel.numel() else 0.0)
    del warm_tau

    opc = build_opcount(grids, wstats, build_ms * 1e-3, plain_s)
    kernels = {k: {"launches_per_step": v[0], "ms_per_step": v[1],
                   "avg_us": 1e3 * v[1] / max(v[0], 1)} for k, v in prof_all.items()}
    kernels[dom] = {"launches_per_step": prof[dom][0] / args.steps,
                    "ms_per_step": prof[dom][1] / args.steps,
                    "avg_us": 1e3 * prof[dom][1] / max(prof[dom][0], 1), "timed_region": True}
    # roofline of the dominant kernel
    node_fields = sum(len(g["m"].sources) * 2 * g["n"] for g in grids)
    if dom in ("k_relax_tau", "k_relax_persist_tau"):
        # per (problem, node): its weight row (|O| doubles) + tau read and written
        alg_step = node_fields * (n_off * 8 + 16)
        per_launch = alg_step / kernels[dom]["launches_per_step"]
        gbs = per_launch / (kernels[dom]["avg_us"] * 1e-6) / 1e9
        traffic = measured_traffic_bytes(dom, "shots")
        roof = {"kernel": dom, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
                "work_per_launch": f"{per_launch:.4g} algorithmic bytes ({n_off} x 8 B weights "
                                   "+ 16 B tau per problem node, over the launches of a step)",
                "avg_launch_us": kernels[dom]["avg_us"],
                "traffic_over_algorithmic": traffic / per_launch if traffic else None}
    else:
        roof = {"kernel": dom, "bound": "fp64", "achieved": None, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": None, "traffic": None}
    st = stats.as_dict()
    res = {
        "metric": METRIC,
        "value": shots / (wall / args.steps),
        "unit": "shots/s ((source, mode) jobs with tau_R + pred + t*, whole step: "
                "surrogate-started per-node cache build + batched trace)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded workloads.config4)",
        "config": {"workload": "batched shots: 128 sources over 4 uneven per-node grids "
                               "(401x201, 801x401, 1201x301, 1701x351 @10 m), qP+qSV, radius 5, "
                               "tau_R + pred + t*, surrogate-started per-node caches",
                   "grids": [[g["m"].nx, g["m"].nz] for g in grids], "sources_per_grid": 32,
                   "modes": [0, 1], "radius": 5, "nodes": sum(g["n"] for g in grids),
                   "parallelism": "single GPU"},
        "breakdown": {
            "build_ms": build_ms, "trace_ms": trace_ms,
            "hamiltonian_solves_per_s_warm": solves / (build_ms * 1e-3),
            "hamiltonian_solves_per_s_plain": solves / plain_s,
            "plain_build_s": plain_s, "surrogate_gain_build": plain_s / (build_ms * 1e-3),
            "unique_solves_per_step": solves,
            "useful_edge_relaxations_per_s_trace": useful / (trace_ms * 1e-3),
            "useful_edge_relaxations_per_s_step": useful / (wall / args.steps),
            "useful_edges_per_step": useful,
            "shots_per_s_trace_only": shots / (trace_ms * 1e-3),
            "graph_replay_trace_s": graph_s,
            "shots_per_s_graph_trace_only": shots / graph_s if graph_s else None,
            "persistent_graph_replay_trace_s": pgraph_s,
            "shots_per_s_persistent_graph_trace_only": shots / pgraph_s if pgraph_s else None,
            "tau_R_rel_surrogate_vs_plain_max": worst, "tau_R_within_1e-4": worst <= 1e-4,
            "same_reachability": same_reach, "warm_status_equals_plain": same_status,
            "warm_stats": wstats, "training": tinfo, "build_opcount": opc,
            "trace_stats_last_step": st,
            "raw_over_useful": {"tau": st["edge_relaxations"][0] / useful,
                                "tree": st["edge_relaxations"][1] / useful},
            "launch": {"tile": [opts.tile_x or 32, opts.tile_z or 32],
                       "push_group": opts.push_group or 2, "launch": LAUNCH_NAMES[opts.launch],
                       "bucket_width": opts.bucket_width, "autotune": tune},
            "kernels": kernels,
        },
        "roofline": roof,
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline_shots(grids, solves, node_fields, shots, opts)
    print(json.dumps(res))


def build_opcount(grids, wstats, warm_s, plain_s, n_sample=32):
    """Algorithmic FP64 work of the per-node builds from an operation count
    of the kernel source (paper_2609_26108_amd.opcount: physics.h and
    solve.h compiled on the host with a counting scalar) on a sample of
    solid nodes of the first grid, per mode: the theta_R sweep per class,
    the plain solve per direction, and the surrogate start's polish per
    direction (from a root offset by 1e-3 / 2e-4 rad, the surrogate's
    typical miss).  Work per step = polished directions x polish cost +
    window samples x sweep-sample cost + plain-path jobs (fallbacks) x
    (sweep + directions x solve); rates over
    the measured build times against the FP64 vector peak; fold-window
    samples count as sweep samples.  Transcendental
    calls (sincos, expm1, atan2) are counted apart and not in the flops."""
    import paper_2609_26108_amd as C
    from paper_2609_26108_amd import opcount
    g = grids[0]
    rows = g["m"].param_rows()
    solid = np.flatnonzero(rows[:, 1] > 0.0)
    pick = solid[np.linspace(0, solid.size - 1, n_sample).astype(int)]
    cls = np.stack([C.chert_class_from_thomsen(*r).as_array() for r in rows[pick]])
    n_solve = len(g["sub"]) // 2
    per = {}
    for mode in (0, 1):
        b = opcount.count(cls, n_dirs=2 * n_solve, n_sweep=g["desc"].n_sweep, mode=mode)["build"]
        per[mode] = b
    mean = {k: 0.5 * (per[0][k] + per[1][k]) for k in
            ("sweep_flops_per_class", "solve_flops_per_direction", "warm_flops_per_direction",
             "sweep_trans_per_class", "solve_trans_per_direction", "warm_trans_per_direction")}
    jobs = sum(2 * gg["n"] for gg in grids)
    plain_job = mean["sweep_flops_per_class"] + n_solve * mean["solve_flops_per_direction"]
    # fold windows: each evaluated sample is one sweep sample's work
    sample = mean["sweep_flops_per_class"] / g["desc"].n_sweep
    warm_flops = (wstats["directions"] * mean["warm_flops_per_direction"] +
                  wstats["window_samples"] * sample + wstats["fallback_jobs"] * plain_job)
    plain_flops = jobs * plain_job
    return {"per_mode": {str(m): per[m] for m in per}, "solved_directions_per_job": n_solve,
            "energy_eval_flops": opcount.count(cls[:1], n_dirs=4, n_sweep=64)["MEV_qP"][
                "energy_eval_flops"],
            "warm_step_flops": warm_flops, "plain_build_flops": plain_flops,
            "warm_tflops": warm_flops / warm_s / 1e12,
            "warm_frac_fp64": warm_flops / warm_s / 1e12 / FP64_PEAK_TFLOPS,
            "plain_tflops": plain_flops / plain_s / 1e12,
            "plain_frac_fp64": plain_flops / plain_s / 1e12 / FP64_PEAK_TFLOPS,
            "note": "counted add/sub/mul/div/sqrt of the source (an FMA = 2); transcendental "
                    "calls apart; sample of solid nodes of the 401x201 grid"}


def cpu_baseline_shots(grids, solves_total, node_fields_total, shots, opts):
    """The CPU oracle as it stands, one core, on a fixed subset of the
    batched-shots step, extrapolated linearly to the whole step: its plain
    cache build of the first 160 solid nodes of the first grid (both modes,
    the star's bins), and its Dijkstra (tau_R, predecessors, t*) for the
    first shot of the first grid in both modes on the GPU-built plain cache.
    Parity is checked on that subset: the oracle's entries against the GPU
    plain cache's, its fields against the GPU's through the plain cache."""
    import torch
    import oracle as O
    O.build(force=False)
    g = grids[0]
    m, n, sub, desc = g["m"], g["n"], g["sub"], g["desc"]
    rows = m.param_rows()
    pick = np.flatnonzero(rows[:, 1] > 0.0)[:160]
    cls = np.stack([O.class_from_thomsen(*r) for r in rows[pick]])
    t0 = time.perf_counter()
    fo, so = O.build_cache_2d(cls, mode_mask=0b011, subset=sub)
    t_cache = time.perf_counter() - t0
    n_solves = _converged(so[:2]) // 2
    import paper_2609_26108_amd as C
    fv, sv = C.cache_views(g["plain"], desc, n)
    fp = fv[:, :2].cpu().numpy()
    sp = sv[:2].cpu().numpy()
    ok = (so[:2] & (1 | 4 | 8)) == 0
    same_status = bool(np.array_equal(sp[:, pick], so[:2]))
    relV = np.abs(fp[0][:, pick][ok] - fo[0, :2][ok]) / np.abs(fo[0, :2][ok])
    # Dijkstra of the first shot, both modes, on the plain cache (the GPU's
    # fields through that cache were computed last, by the plain batch)
    t_trace, bitwise = 0.0, True
    src = m.sources[0]
    for mode in (0, 1):
        V, A, S = fp[0][mode], fp[1][mode], sp[mode]
        t0 = time.perf_counter()
        o = O.trace_2d(m.nx, m.nz, m.hx, m.hz, None, m.radius, V, A, S, src, 360, sub, False)
        t_trace += time.perf_counter() - t0
        out = g["outs"][mode]
        for gk, okk in (("tau_r", "tauR"), ("tstar", "tstar"), ("pred_p", "predP")):
            bitwise &= bool(np.array_equal(out[gk][0].cpu().numpy(), o[okk]))
    cache_rate = n_solves / t_cache                 # unique solves per second
    trace_rate = 2 * n / t_trace                    # problem nodes per second
    t_step = solves_total / cache_rate + node_fields_total / trace_rate
    # the same oracle on every host core over independent tasks (node chunks
    # of the cache sample; one shot and mode per Dijkstra); the oracle's C
    # calls release the interpreter lock, so threads run them in parallel
    from concurrent.futures import ThreadPoolExecutor
    T = max(1, min(16, os.cpu_count() or 1))
    chunks = [c for c in np.array_split(np.arange(len(pick)), T) if c.size]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(T) as ex:
        list(ex.map(lambda c: O.build_cache_2d(cls[c], mode_mask=0b011, subset=sub), chunks))
    t_cache_T = time.perf_counter() - t0
    tasks = [(m.sources[k % len(m.sources)], k % 2) for k in range(T)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(T) as ex:
        list(ex.map(lambda t: O.trace_2d(m.nx, m.nz, m.hx, m.hz, None, m.radius, fp[0][t[1]],
                                         fp[1][t[1]], sp[t[1]], t[0], 360, sub, False), tasks))
    t_trace_T = time.perf_counter() - t0
    t_step_T = (solves_total / (n_solves / t_cache_T) +
                node_fields_total / (len(tasks) * n / t_trace_T))
    return {"value": shots / t_step, "unit": "shots/s (extrapolated whole step)", "cores": 1,
            "all_cores": {"value": shots / t_step_T, "cores": T,
                          "sample": f"the cache sample split over {len(chunks)} threads; "
                                    f"{len(tasks)} single-shot Dijkstras (tau_R, pred, t*) at once"},
            "kind": "oracle",
            "sample": f"plain cache build of {len(pick)} solid nodes of the 401x201 grid (qP+qSV, "
                      "80 star bins) and Dijkstra (tau_R, pred, t*) of its first shot in both "
                      "modes; extrapolated linearly (cache by unique solves, trace by problem "
                      "nodes) to the 256-job step",
            "extrapolated": True, "sample_cache_s": t_cache, "sample_trace_s": t_trace,
            "cache_solves_per_s": cache_rate, "trace_problem_nodes_per_s": trace_rate,
            "extrapolated_step_s": t_step,
            "parity_on_sample": {"cache_status_equal": same_status,
                                 "cache_V_rel_max": float(relV.max()) if relV.size else 0.0,
                                 "fields_bitwise": bitwise},
            "cpu_count": os.cpu_count()}


ABL_STEPS = (720, 360, 180, 36)   # 0.5, 1, 2 and 10 degree angular sampling
ABL_RADII = (2, 3, 4, 5, 6)


def _misfit(a, ref):
    """RMS and max of tau - tau_ref over nodes reachable in both [s], and the
    max relative difference."""
    fin = torch_isfinite(a) & torch_isfinite(ref)
    d = (a[fin] - ref[fin])
    rel = d.abs() / ref[fin].abs().clamp_min(1e-300)
    return {"rms_ms": 1e3 * float(d.pow(2).mean().sqrt().item()),
            "max_abs_ms": 1e3 * float(d.abs().max().item()),
            "max_rel": float(rel.max().item()),
            "reachable": int(fin.sum().item())}


def torch_isfinite(t):
    import torch
    return torch.isfinite(t)


def run_ablation(args):
    """Angular-step and star-radius ablations (the paper's angular-sampling
    and node-density study): angular steps 0.5, 1, 2 and 10 degrees and
    forward-star radii 2..6, on the layered model (class caches, qP/qSV/qSH)
    and on the structurally complex model (per-node surrogate-started caches
    on the star's bins, qSV).  For every setting: cache build and trace
    times, and the tau_R misfit against the finest setting (0.5 degree,
    radius 6)."""
    import torch
    import paper_2609_26108_amd as C
    import workloads as W
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    res = {"metric": METRIC, "workload": "ablation", "n_gpus": 1, "dtype": "f64",
           "data": "synthetic (seeded workloads.config2, workloads.complex_2d)",
           "config": {"workload": "angular step {0.5, 1, 2, 10} deg x star radius {2..6}; "
                                  "layered 401x201 @5 m (class caches) and complex 1701x351 "
                                  "@10 m (per-node caches)", "steps_deg": [360 / n for n in ABL_STEPS],
                      "radii": list(ABL_RADII), "reference": "0.5 deg, radius 6"}}
    # layered model, class caches: one cache per step, one trace per radius
    m = W.config2()
    K = len(m.layers)
    cls = torch.from_numpy(np.stack([C.chert_class_from_thomsen(*L.thomsen_args()).as_array()
                                     for L in m.layers])).to(dev)
    cid = torch.from_numpy(m.class_id.reshape(-1).astype(np.int32)).to(dev)
    n = m.n_nodes
    taus, lay2 = {}, {}
    for nd in ABL_STEPS:
        desc = C.cache_desc(n_dirs=nd, modes=m.modes)
        lay = C.chert_cache_layout_of(desc, K)
        cache = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=dev)
        ws = torch.empty(max(C.chert_build_cache_workspace_bytes(desc, K), 1), dtype=torch.uint8,
                         device=dev)
        C.chert_build_cache(desc, cls, K, cache, ws, stream=stream)  # warm-up
        ev = _events(torch, stream)
        C.chert_build_cache(desc, cls, K, cache, ws, stream=stream)
        t_build = _elapsed(torch, ev, stream)
        for R in ABL_RADII:
            grid = C.make_grid(m.nx, m.nz, m.hx, m.hz, R, cid)
            b = C.Batch()
            outs = {}
            for mode in m.modes:
                outs[mode] = torch.empty((1, n), dtype=torch.float64, device=dev)
                b.add(desc, cache, K, grid, mode, m.sources, tau_r=outs[mode])
            o = C.trace_opts(C.OUT_TAU_R)
            tws = torch.empty(C.chert_trace_batch_workspace_bytes(b, o), dtype=torch.uint8,
                              device=dev)
            C.chert_trace_batch(b, o, tws, stream=stream)
            ev = _events(torch, stream)
            C.chert_trace_batch(b, o, tws, stream=stream)
            t_trace = _elapsed(torch, ev, stream)
            taus[(nd, R)] = {mode: outs[mode][0].clone() for mode in m.modes}
            lay2[(nd, R)] = {"build_s": t_build, "trace_s": t_trace}
    ref = taus[(720, 6)]
    res["layered"] = {f"{360 / nd:g}deg_R{R}": {
        **lay2[(nd, R)],
        "misfit": {str(mode): _misfit(taus[(nd, R)][mode], ref[mode]) for mode in m.modes}}
        for nd in ABL_STEPS for R in ABL_RADII}
    del taus

    # structurally complex model, per-node caches (surrogate-started)
    blob, tinfo = train_surrogate(args, dev, stream)
    res["training"] = tinfo
    mc = W.complex_2d()
    rows = mc.param_rows()
    nn = rows.shape[0]
    ccls = torch.empty((nn, 13), dtype=torch.float64, device=dev)
    C.chert_classes_from_thomsen(torch.from_numpy(rows).to(dev), ccls)
    mode = mc.modes[0]
    taus, out = {}, {}
    for nd in ABL_STEPS:
        for R in ABL_RADII:
            sub = C.star_subset(R, mc.hx, mc.hz, nd)
            desc = C.cache_desc(n_dirs=nd, modes=(mode,), subset=sub)
            lay = C.chert_cache_layout_of(desc, nn)
            cache = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=dev)
            wws = torch.empty(C.chert_build_cache_surrogate_workspace_bytes(desc, nn),
                              dtype=torch.uint8, device=dev)
            wst = torch.zeros(C.WARM_NSTATS, dtype=torch.int64, device=dev)
            ev = _events(torch, stream)
            C.chert_build_cache_surrogate(desc, ccls, nn, blob, cache, wws, wst, stream=stream)
            t_build = _elapsed(torch, ev, stream)
            del wws
            grid = C.make_grid(mc.nx, mc.nz, mc.hx, mc.hz, R, None)
            tr = torch.empty((1, nn), dtype=torch.float64, device=dev)
            o = C.trace_opts(C.OUT_TAU_R)
            tws = torch.empty(C.chert_trace_workspace_bytes(desc, nn, grid, 1, o),
                              dtype=torch.uint8, device=dev)
            C.chert_trace_field(desc, cache, nn, grid, mode, mc.sources, o, tr, None, None, None,
                                None, tws, stream=stream)
            ev = _events(torch, stream)
            C.chert_trace_field(desc, cache, nn, grid, mode, mc.sources, o, tr, None, None, None,
                                None, tws, stream=stream)
            t_trace = _elapsed(torch, ev, stream)
            del tws, cache
            taus[(nd, R)] = tr[0].clone()
            w = dict(zip(C.WARM_STATS, wst.cpu().numpy().tolist()))
            out[(nd, R)] = {"columns": int(len(sub)), "build_s": t_build, "trace_s": t_trace,
                            "fallback_jobs": w["fallback_jobs"]}
    ref = taus[(720, 6)]
    res["complex"] = {f"{360 / nd:g}deg_R{R}": {**out[(nd, R)],
                                                "misfit": _misfit(taus[(nd, R)], ref)}
                      for nd in ABL_STEPS for R in ABL_RADII}
    # the paper's cost statement: the 1-degree cache costs about half the
    # 0.5-degree one (class caches: the number of solved directions)
    res["layered_build_ratio_1deg_over_0p5deg"] = (res["layered"]["1deg_R5"]["build_s"] /
                                                   res["layered"]["0.5deg_R5"]["build_s"])
    res["value"] = res["complex"]["1deg_R5"]["misfit"]["rms_ms"]
    res["unit"] = "ms RMS tau_R misfit of the 1-degree, radius-5 per-node trace against 0.5 deg / R 6"
    res["higher_is_better"] = False
    print(json.dumps(res))


LOCAL_FINE = 360000  # slowness samples of the timed local sweep (0.001 degree)


def rock_layer1_class():
    """Layer 1 of the paper's rock-property table (the medium of its local
    kernel benchmark) as a class row: moduli in m^2/s^2, Q per component,
    vertical symmetry axis."""
    with open(os.path.join(ROOT, "tests", "golden", "rock_table.txt")) as f:
        rows = [[float(x) for x in ln.split()[1:]] for ln in f
                if ln.strip() and not ln.startswith("#")]
    r = rows[0]
    return np.array([v * 1e6 for v in r[:5]] + r[5:10] + [2300.0, 0.0, 0.0])


def _angle_sweep_stats(f, st, mode, cols):
    """Range and smoothness of one mode's cache columns `cols` (adjacent
    samples): theta_I range and its largest step [deg], the largest relative
    step of V and A, and the status counts."""
    bad = 1 | 4 | 8 | 16  # NO_BRACKET, FLUID, NONPHYS, NOCONV
    s = st[mode, 0, cols]
    ok = (s & bad) == 0
    thi = np.degrees(f[6, mode, 0, cols])
    V, A = f[0, mode, 0, cols], f[1, mode, 0, cols]
    pair = ok[1:] & ok[:-1]
    out = {"samples": int(len(cols)), "usable": int(ok.sum()),
           "ill": int(((s & 2) != 0).sum()), "noconv": int(((s & 16) != 0).sum()),
           "no_bracket": int(((s & 1) != 0).sum())}
    if ok.any():
        out["thetaI_deg"] = [float(thi[ok].min()), float(thi[ok].max())]
    if pair.any():
        out["max_step_thetaI_deg"] = float(np.abs(np.diff(thi))[pair].max())
        out["max_rel_step_V"] = float((np.abs(np.diff(V)) / V[:-1])[pair].max())
        out["max_rel_step_A"] = float((np.abs(np.diff(A)) / np.abs(A[:-1]))[pair].max())
    return out


def run_local(args):
    """The local kernel benchmark (the paper's OEV-versus-MEV sweep on layer
    1 of its rock table, eqs 12-14 and 26) and the cache-sampling comparison
    it motivates: for each reading, the slowness-sampled cache (eq 26 at every
    real slowness angle) and the ray-direction cache at 1 degree, with the
    theta_I range and the smoothness of theta_I, V and A over 0-90 degrees;
    then the slowness sweep at 0.001 degree timed (Hamiltonian solves/s),
    and traveltimes of the layered model through slowness-sampled and
    ray-direction caches against each other."""
    import torch
    import paper_2609_26108_amd as C
    import workloads as W
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    cls = torch.from_numpy(rock_layer1_class()[None]).to(dev)
    modes = (0, 1, 2)
    names = {0: "qP", 1: "qSV", 2: "qSH"}
    res = {"metric": METRIC, "workload": "local", "n_gpus": 1, "dtype": "f64",
           "data": "layer 1 of the paper's rock-property table (tests/golden/rock_table.txt); "
                   "seeded workloads.config2 for the traveltime comparison",
           "config": {"workload": "local sweep on rock layer 1: 1-degree caches (slowness- and "
                                  "ray-sampled, MEV and OEV) and a 0.001-degree slowness sweep; "
                                  "layered 401x201 @5 m traveltimes through both samplings",
                      "fine_samples": LOCAL_FINE}}
    sweep = {}
    for kname, kern in (("MEV", C.KERNEL_MEV), ("OEV", C.KERNEL_OEV)):
        for sname, samp in (("slowness", C.SAMPLE_SLOWNESS), ("ray", C.SAMPLE_RAY)):
            desc = C.cache_desc(n_dirs=360, modes=modes, kernel=kern, sampling=samp)
            lay = C.chert_cache_layout_of(desc, 1)
            cache = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=dev)
            ws = torch.empty(max(C.chert_build_cache_workspace_bytes(desc, 1), 1),
                             dtype=torch.uint8, device=dev)
            C.chert_build_cache(desc, cls, 1, cache, ws, stream=stream)
            torch.cuda.synchronize()
            f, st = C.cache_views(cache, desc, 1)
            f, st = f.cpu().numpy(), st.cpu().numpy()
            sweep[f"{kname}_{sname}"] = {names[m]: _angle_sweep_stats(f, st, m, np.arange(91))
                                         for m in modes}
    res["sweep_1deg_0_90"] = sweep

    timing = {}
    for kname, kern in (("MEV", C.KERNEL_MEV), ("OEV", C.KERNEL_OEV)):
        desc = C.cache_desc(n_dirs=LOCAL_FINE, modes=modes, kernel=kern,
                            sampling=C.SAMPLE_SLOWNESS)
        lay = C.chert_cache_layout_of(desc, 1)
        cache = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=dev)
        ws = torch.empty(1, dtype=torch.uint8, device=dev)
        C.chert_build_cache(desc, cls, 1, cache, ws, stream=stream)  # warm-up
        t = []
        for _ in range(max(args.steps, 1)):
            ev = _events(torch, stream)
            C.chert_build_cache(desc, cls, 1, cache, ws, stream=stream)
            t.append(_elapsed(torch, ev, stream))
        ts = float(np.median(t))
        _, st = C.cache_views(cache, desc, 1)
        st = st.cpu().numpy()
        timing[kname] = {"build_s": ts, "solves_per_s": 3 * LOCAL_FINE / ts,
                         "usable": int(((st & (1 | 4 | 8 | 16)) == 0).sum())}
    res["fine_sweep"] = timing

    # traveltimes through both samplings (MEV, 1 degree, class caches)
    m = W.config2()
    K = len(m.layers)
    lcls = torch.from_numpy(np.stack([C.chert_class_from_thomsen(*L.thomsen_args()).as_array()
                                      for L in m.layers])).to(dev)
    cid = torch.from_numpy(m.class_id.reshape(-1).astype(np.int32)).to(dev)
    grid = C.make_grid(m.nx, m.nz, m.hx, m.hz, m.radius, cid)
    taus = {}
    for sname, samp in (("slowness", C.SAMPLE_SLOWNESS), ("ray", C.SAMPLE_RAY)):
        desc = C.cache_desc(n_dirs=360, modes=m.modes, sampling=samp)
        lay = C.chert_cache_layout_of(desc, K)
        cache = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=dev)
        ws = torch.empty(max(C.chert_build_cache_workspace_bytes(desc, K), 1), dtype=torch.uint8,
                         device=dev)
        C.chert_build_cache(desc, lcls, K, cache, ws, stream=stream)
        ev = _events(torch, stream)
        C.chert_build_cache(desc, lcls, K, cache, ws, stream=stream)
        tb = _elapsed(torch, ev, stream)
        b = C.Batch()
        outs = {}
        for mode in m.modes:
            outs[mode] = (torch.empty((1, m.n_nodes), dtype=torch.float64, device=dev),
                          torch.empty((1, m.n_nodes), dtype=torch.float64, device=dev))
            b.add(desc, cache, K, grid, mode, m.sources, tau_r=outs[mode][0],
                  tau_i=outs[mode][1])
        o = C.trace_opts(C.OUT_TAU_R | C.OUT_TAU_I)
        tws = torch.empty(C.chert_trace_batch_workspace_bytes(b, o), dtype=torch.uint8,
                          device=dev)
        C.chert_trace_batch(b, o, tws, stream=stream)
        ev = _events(torch, stream)
        C.chert_trace_batch(b, o, tws, stream=stream)
        tt = _elapsed(torch, ev, stream)
        taus[sname] = ({mode: (outs[mode][0][0].clone(), outs[mode][1][0].clone())
                        for mode in m.modes}, tb, tt)
    a, b_ = taus["slowness"][0], taus["ray"][0]
    res["layered_slowness_vs_ray"] = {
        "build_s": {"slowness": taus["slowness"][1], "ray": taus["ray"][1]},
        "trace_s": {"slowness": taus["slowness"][2], "ray": taus["ray"][2]},
        "tauR_misfit": {names[md]: _misfit(a[md][0], b_[md][0]) for md in m.modes},
        "tauI_misfit": {names[md]: _misfit(a[md][1], b_[md][1]) for md in m.modes}}

    if not args.no_cpu:
        import oracle as O
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < 10.0:
            O.build_cache_slow_2d(rock_layer1_class()[:13], n=3600, mode_mask=0b111)
            reps += 1
        el = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": reps * 3 * 3600 / el, "unit": "Hamiltonian solves/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"{reps} slowness-sampled builds of rock layer 1, "
                                         "3 modes x 3600 samples (MEV)"}
    res["value"] = timing["MEV"]["solves_per_s"]
    res["unit"] = "Hamiltonian solves/s (slowness-sampled MEV, rock layer 1, 3 modes)"
    res["higher_is_better"] = True
    print(json.dumps(res))


CELL_BUCKETS = (0.0, 4.0, 16.0, 64.0)


def cell_pairs(ncx, ncz, cn):
    """Directed segments of the cell network: ordered pairs of distinct
    boundary nodes per cell (a pair along an edge shared by two cells is
    counted once per cell)."""
    nb = 4 * cn
    return ncx * ncz * nb * (nb - 1)


def run_cells(args):
    """The paper's cell network (nodes on cell edges, every boundary pair of
    a cell a segment; eqs 23-24, 27-32) on the layered model: cells of 5x5
    lattice intervals over the 401x201 lattice at 5 m (80x40 cells), class
    caches at 1 degree, qP/qSV/qSH from the surface source.  Timed per mode
    with every woken cell per round and with block-ordered rounds of several
    widths; traveltimes compared with the radius-5 forward star on the same
    lattice (the node density study's comparison at matched angular
    coverage)."""
    import torch
    import paper_2609_26108_amd as C
    import workloads as W
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    m = W.config2()
    cn = 5
    ncx, ncz = (m.nx - 1) // cn, (m.nz - 1) // cn
    K = len(m.layers)
    cls = torch.from_numpy(np.stack([C.chert_class_from_thomsen(*L.thomsen_args()).as_array()
                                     for L in m.layers])).to(dev)
    desc = C.cache_desc(n_dirs=360, modes=m.modes)
    lay = C.chert_cache_layout_of(desc, K)
    cache = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=dev)
    ws = torch.empty(max(C.chert_build_cache_workspace_bytes(desc, K), 1), dtype=torch.uint8,
                     device=dev)
    C.chert_build_cache(desc, cls, K, cache, ws, stream=stream)
    cid = torch.from_numpy(m.class_id.reshape(-1).astype(np.int32)).to(dev)
    cg = C.make_cell_grid(ncx, ncz, cn, m.hx, m.hz, cid)
    n = m.n_nodes
    ix = np.arange(m.nx)[None, :]
    iz = np.arange(m.nz)[:, None]
    node_mask = torch.from_numpy(((ix % cn == 0) | (iz % cn == 0)).reshape(-1)).to(dev)
    pairs = cell_pairs(ncx, ncz, cn)
    res = {"metric": METRIC, "workload": "cells", "n_gpus": 1, "dtype": "f64",
           "data": "synthetic (seeded workloads.config2)",
           "config": {"workload": f"cell network {ncx}x{ncz} cells of {cn}x{cn} intervals on "
                                  "the 5-layer 401x201 lattice @5 m, 1-degree class caches, "
                                  "qP/qSV/qSH, one surface source",
                      "network_nodes": int(node_mask.sum().item()), "segments": pairs}}
    outs = C.OUT_ALL
    per = {}
    taus = {}
    for bw in CELL_BUCKETS:
        row = {}
        for mode in m.modes:
            st = C.TraceStats()
            o = C.trace_opts(outs, bucket_width=bw, stats=st)
            t = {k: torch.empty((1, n), dtype=dt, device=dev) for k, dt in
                 (("tr", torch.float64), ("ti", torch.float64), ("ts", torch.float64),
                  ("pp", torch.int32), ("pa", torch.int32))}
            tws = torch.empty(C.chert_trace_cells_workspace_bytes(desc, K, cg, 1, o),
                              dtype=torch.uint8, device=dev)
            C.chert_trace_cells(desc, cache, K, cg, mode, m.sources, o, t["tr"], t["ti"],
                                t["ts"], t["pp"], t["pa"], tws, stream=stream)
            times = []
            for _ in range(max(args.steps, 1)):
                ev = _events(torch, stream)
                C.chert_trace_cells(desc, cache, K, cg, mode, m.sources, o, t["tr"], t["ti"],
                                    t["ts"], t["pp"], t["pa"], tws, stream=stream)
                times.append(_elapsed(torch, ev, stream))
            ts = float(np.median(times))
            # the traveltime phase alone (no predecessors)
            st2 = C.TraceStats()
            o2 = C.trace_opts(C.OUT_TAU_R | C.OUT_TAU_I, bucket_width=bw, stats=st2)
            C.chert_prof_enable(True)
            C.chert_trace_cells(desc, cache, K, cg, mode, m.sources, o2, t["tr"], t["ti"],
                                None, None, None, tws, stream=stream)
            torch.cuda.synchronize()
            prof = C.chert_prof_read()
            C.chert_prof_enable(False)
            relax_s = prof.get("k_cell_relax", (0, 0.0))[1] * 1e-3
            row[str(mode)] = {"s": ts, "rounds": st.rounds[0], "bfs_levels": st.rounds[1],
                              "cell_visits": st.tile_visits[0],
                              "pair_relaxations": st.edge_relaxations[0],
                              "relax_kernel_s": relax_s,
                              "relax_kernel_pairs": st2.edge_relaxations[0],
                              "pair_relaxations_per_s": st2.edge_relaxations[0] / max(relax_s, 1e-12)}
            if bw == 0.0:
                taus[mode] = t["tr"][0].clone()
        per[f"bucket_{bw:g}"] = row
    res["modes"] = per
    # forward star of radius 5 on the same lattice, at the network's nodes
    grid = C.make_grid(m.nx, m.nz, m.hx, m.hz, 5, cid)
    o = C.trace_opts(C.OUT_TAU_R)
    cmp = {}
    for mode in m.modes:
        tr = torch.empty((1, n), dtype=torch.float64, device=dev)
        tws = torch.empty(C.chert_trace_workspace_bytes(desc, K, grid, 1, o), dtype=torch.uint8,
                          device=dev)
        C.chert_trace_field(desc, cache, K, grid, mode, m.sources, o, tr, None, None, None, None,
                            tws, stream=stream)
        torch.cuda.synchronize()
        cmp[str(mode)] = _misfit(taus[mode][node_mask], tr[0][node_mask])
    res["cells_vs_star_R5_tauR"] = cmp
    # a batch of surface sources per call: the rounds of all problems share
    # the launches
    n_batch = 16
    bsrc = [int(x) for x in np.linspace(0, ncx, n_batch).astype(int) * cn]
    bres = {}
    for bw in (0.0, 16.0):
        tot = rk_s = 0.0
        rk_p = rk_n = 0
        for mode in m.modes:
            o = C.trace_opts(outs, bucket_width=bw)
            t = {k: torch.empty((n_batch, n), dtype=dt, device=dev) for k, dt in
                 (("tr", torch.float64), ("ti", torch.float64), ("ts", torch.float64),
                  ("pp", torch.int32), ("pa", torch.int32))}
            tws = torch.empty(C.chert_trace_cells_workspace_bytes(desc, K, cg, n_batch, o),
                              dtype=torch.uint8, device=dev)
            C.chert_trace_cells(desc, cache, K, cg, mode, bsrc, o, t["tr"], t["ti"], t["ts"],
                                t["pp"], t["pa"], tws, stream=stream)
            ev = _events(torch, stream)
            C.chert_trace_cells(desc, cache, K, cg, mode, bsrc, o, t["tr"], t["ti"], t["ts"],
                                t["pp"], t["pa"], tws, stream=stream)
            tot += _elapsed(torch, ev, stream)

            def call(st, o_bw=bw, t=t, tws=tws, mode=mode):
                C.chert_trace_cells(desc, cache, K, cg, mode, bsrc,
                                    C.trace_opts(outs, bucket_width=o_bw, stats=st), t["tr"],
                                    t["ti"], t["ts"], t["pp"], t["pa"], tws, stream=stream)
            ks, kp, kn = _batch_relax_profile(C, torch, call, "k_cell_relax")
            rk_s += ks
            rk_p += kp
            rk_n += kn
        bres[f"bucket_{bw:g}"] = {"s_all_modes": tot,
                                  "fields_per_s": len(m.modes) * n_batch / tot,
                                  "relax_kernel_s": rk_s, "relax_kernel_pairs": rk_p,
                                  "relax_kernel_launches": rk_n}
    res["batch_16_sources"] = bres
    res["value"] = max(v["fields_per_s"] for v in bres.values())
    res["unit"] = ("fields/s (tau_R, tau_I, predecessors and t* per source and mode, "
                   "16 sources per call, cell network)")
    res["higher_is_better"] = True
    # ALU roofline of the pair relaxation in the batch the value is quoted
    # on: one add and one compare per pair
    dom = max(bres.values(), key=lambda v: v["fields_per_s"])
    ach = 2.0 * dom["relax_kernel_pairs"] / max(dom["relax_kernel_s"], 1e-12) / 1e12
    res["roofline"] = {"bound": "alu", "achieved": ach, "peak": FP64_VALU_PEAK_TOPS,
                       "unit": "TFLOP/s", "frac": ach / FP64_VALU_PEAK_TOPS, "traffic": None,
                       "kernel": "k_cell_relax",
                       "avg_launch_us": 1e6 * dom["relax_kernel_s"] / max(dom["relax_kernel_launches"], 1)}
    if not args.no_cpu:
        import oracle as O
        cls_np = np.stack([O.class_from_thomsen(*L.thomsen_args()) for L in m.layers])
        f, st = O.build_cache_2d(cls_np, n_dirs=360, mode_mask=0b001)
        t0 = time.perf_counter()
        O.trace_cells_2d(ncx, ncz, cn, m.hx, m.hz, m.class_id, f[:, 0], st[0], m.sources[0])
        el = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": 1.0 / el, "unit": "fields/s (all five outputs, qP)",
                               "cores": 1, "kind": "oracle",
                               "sample": "one qP field of the same network (node Dijkstra, "
                                         "predecessors, t*)"}
    print(json.dumps(res))


def run_blocks(args):
    """The compact 3D TTI model on the block network (the cell network in
    3D): 18 x 18 x 4 blocks of 160 m, block edges of 3 intervals (a
    55 x 55 x 13 lattice at 53.3 m), four undulating layers tilted 25 degrees
    with seeded azimuths, a 41,253-direction Fibonacci cache of qP and qSV,
    the centre surface source.  Times the cache build and one trace per mode
    (all five outputs) at several ordering widths, then a batch of 16
    surface sources per call."""
    import torch
    import paper_2609_26108_amd as C
    import workloads as W
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    m = W.blocks_3d()
    K = len(m.layers)
    NX, NY, NZ = m.lattice
    n = NX * NY * NZ
    cls = torch.from_numpy(np.stack([C.chert_class_from_thomsen(*L.thomsen_args()).as_array()
                                     for L in m.layers])).to(dev)
    desc = C.cache_desc(dim=3, n_dirs=m.n_dirs, modes=m.modes)
    lay = C.chert_cache_layout_of(desc, K)
    cache = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=dev)
    cws = torch.empty(max(C.chert_build_cache_workspace_bytes(desc, K), 1), dtype=torch.uint8,
                      device=dev)
    C.chert_build_cache(desc, cls, K, cache, cws, stream=stream)
    builds = []
    for _ in range(3):
        ev = _events(torch, stream)
        C.chert_build_cache(desc, cls, K, cache, cws, stream=stream)
        builds.append(_elapsed(torch, ev, stream))
    cid = torch.from_numpy(m.class_id.reshape(-1).astype(np.int32)).to(dev)
    bg = C.make_block_grid(m.ncx, m.ncy, m.ncz, m.block_n, m.h, m.h, m.h, cid)
    cn = m.block_n
    ix = np.arange(NX)[None, None, :]
    iy = np.arange(NY)[None, :, None]
    iz = np.arange(NZ)[:, None, None]
    n_nodes = int(((ix % cn == 0) | (iy % cn == 0) | (iz % cn == 0)).sum())
    face = (cn + 1) ** 3 - (cn - 1) ** 3
    res = {"metric": METRIC, "workload": "blocks", "n_gpus": 1, "dtype": "f64",
           "data": "synthetic (seeded workloads.blocks_3d)",
           "config": {"workload": f"block network {m.ncx}x{m.ncy}x{m.ncz} blocks of 160 m, "
                                  f"{cn} intervals per edge ({NX}x{NY}x{NZ} lattice), 4 tilted "
                                  "TTI layers, 41253-direction cache, qP/qSV, centre source",
                      "network_nodes": n_nodes,
                      "segments": m.ncx * m.ncy * m.ncz * face * (face - 1),
                      "cache_build_s": float(np.median(builds))}}
    outs = C.OUT_ALL

    def bufs(S):
        return {k: torch.empty((S, n), dtype=dt, device=dev) for k, dt in
                (("tr", torch.float64), ("ti", torch.float64), ("ts", torch.float64),
                 ("pp", torch.int32), ("pa", torch.int32))}

    per = {}
    for bw in (0.0, 4.0, 16.0):
        row = {}
        for mode in m.modes:
            st = C.TraceStats()
            o = C.trace_opts(outs, bucket_width=bw, stats=st)
            t = bufs(1)
            tws = torch.empty(C.chert_trace_blocks_workspace_bytes(desc, K, bg, 1, o),
                              dtype=torch.uint8, device=dev)
            C.chert_trace_blocks(desc, cache, K, bg, mode, m.sources, o, t["tr"], t["ti"],
                                 t["ts"], t["pp"], t["pa"], tws, stream=stream)
            times = []
            for _ in range(max(args.steps, 1)):
                ev = _events(torch, stream)
                C.chert_trace_blocks(desc, cache, K, bg, mode, m.sources, o, t["tr"], t["ti"],
                                     t["ts"], t["pp"], t["pa"], tws, stream=stream)
                times.append(_elapsed(torch, ev, stream))
            st2 = C.TraceStats()
            o2 = C.trace_opts(C.OUT_TAU_R | C.OUT_TAU_I, bucket_width=bw, stats=st2)
            C.chert_prof_enable(True)
            C.chert_trace_blocks(desc, cache, K, bg, mode, m.sources, o2, t["tr"], t["ti"],
                                 None, None, None, tws, stream=stream)
            torch.cuda.synchronize()
            prof = C.chert_prof_read()
            C.chert_prof_enable(False)
            relax_s = prof.get("k_block_relax", (0, 0.0))[1] * 1e-3
            tr0 = t["tr"][0]
            far = tr0[torch.isfinite(tr0)].max().item()  # interior lattice points stay +inf
            row[str(mode)] = {"s": float(np.median(times)), "rounds": st.rounds[0],
                              "bfs_levels": st.rounds[1], "block_visits": st.tile_visits[0],
                              "pair_relaxations": st.edge_relaxations[0],
                              "relax_kernel_s": relax_s,
                              "relax_kernel_pairs": st2.edge_relaxations[0],
                              "max_tau_R_s": far}
        per[f"bucket_{bw:g}"] = row
    res["modes"] = per
    # raypaths (eqs 25, 33-34) of the centre shot to the 361 surface
    # receivers, both fields, from the last traced mode's predecessors
    pp, pa = t["pp"][0].cpu().numpy(), t["pa"][0].cpu().numpy()
    t0 = time.perf_counter()
    lens = [len(C.chert_extract_raypath(pr, m.sources[0], r)) for pr in (pp, pa)
            for r in m.receivers]
    res["raypaths"] = {"receivers": len(m.receivers), "paths": len(lens),
                       "mean_nodes": float(np.mean(lens)), "max_nodes": int(np.max(lens)),
                       "host_s": time.perf_counter() - t0}
    n_batch = 16
    rng = np.random.default_rng(16)
    surf = [ix_ + NX * iy_ for iy_ in range(0, NY, cn) for ix_ in range(0, NX, cn)]
    bsrc = [int(x) for x in rng.choice(surf, n_batch, replace=False)]
    bres = {}
    for bw in (0.0, 4.0):
        tot = rk_s = 0.0
        rk_p = rk_n = 0
        for mode in m.modes:
            o = C.trace_opts(outs, bucket_width=bw)
            t = bufs(n_batch)
            tws = torch.empty(C.chert_trace_blocks_workspace_bytes(desc, K, bg, n_batch, o),
                              dtype=torch.uint8, device=dev)
            C.chert_trace_blocks(desc, cache, K, bg, mode, bsrc, o, t["tr"], t["ti"], t["ts"],
                                 t["pp"], t["pa"], tws, stream=stream)
            ev = _events(torch, stream)
            C.chert_trace_blocks(desc, cache, K, bg, mode, bsrc, o, t["tr"], t["ti"], t["ts"],
                                 t["pp"], t["pa"], tws, stream=stream)
            tot += _elapsed(torch, ev, stream)

            def call(st, o_bw=bw, t=t, tws=tws, mode=mode):
                C.chert_trace_blocks(desc, cache, K, bg, mode, bsrc,
                                     C.trace_opts(outs, bucket_width=o_bw, stats=st), t["tr"],
                                     t["ti"], t["ts"], t["pp"], t["pa"], tws, stream=stream)
            ks, kp, kn = _batch_relax_profile(C, torch, call, "k_block_relax")
            rk_s += ks
            rk_p += kp
            rk_n += kn
        bres[f"bucket_{bw:g}"] = {"s_all_modes": tot,
                                  "fields_per_s": len(m.modes) * n_batch / tot,
                                  "relax_kernel_s": rk_s, "relax_kernel_pairs": rk_p,
                                  "relax_kernel_launches": rk_n}
    res["batch_16_sources"] = bres
    res["value"] = max(v["fields_per_s"] for v in bres.values())
    res["unit"] = ("fields/s (tau_R, tau_I, predecessors and t* per source and mode, "
                   "16 sources per call, block network)")
    res["higher_is_better"] = True
    # ALU roofline of the pair relaxation in the batch the value is quoted on
    dom = max(bres.values(), key=lambda v: v["fields_per_s"])
    ach = 2.0 * dom["relax_kernel_pairs"] / max(dom["relax_kernel_s"], 1e-12) / 1e12
    res["roofline"] = {"bound": "alu", "achieved": ach, "peak": FP64_VALU_PEAK_TOPS,
                       "unit": "TFLOP/s", "frac": ach / FP64_VALU_PEAK_TOPS, "traffic": None,
                       "kernel": "k_block_relax",
                       "avg_launch_us": 1e6 * dom["relax_kernel_s"] / max(dom["relax_kernel_launches"], 1)}
    if not args.no_cpu:
        import oracle as O
        cls_np = np.stack([O.class_from_thomsen(*L.thomsen_args()) for L in m.layers])
        f, st = O.build_cache_3d(cls_np, N=400, mode_mask=0b001)
        t0 = time.perf_counter()
        O.trace_blocks_3d(m.ncx, m.ncy, m.ncz, cn, m.h, m.h, m.h, m.class_id, f[0, 0], f[1, 0],
                          st[0], m.sources[0], N=400)
        el = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": 1.0 / el, "unit": "fields/s (all five outputs, qP)",
                               "cores": 1, "kind": "oracle",
                               "sample": "one qP field of the same network on a 400-direction "
                                         "oracle cache (node Dijkstra, predecessors, t*)"}
    print(json.dumps(res))


def rock_table_classes():
    """The four layers of the paper's rock-property table as class rows
    (moduli in m^2/s^2, Q per component, vertical symmetry axis)."""
    with open(os.path.join(ROOT, "tests", "golden", "rock_table.txt")) as f:
        rows = [[float(x) for x in ln.split()[1:]] for ln in f
                if ln.strip() and not ln.startswith("#")]
    return np.array([[v * 1e6 for v in r[:5]] + r[5:10] + [2300.0, 0.0, 0.0] for r in rows])


def run_mspm(args):
    """The paper's controlled field-scale benchmark, CHERT against MSPM on
    the same network: the four layers of its rock-property table as flat
    VTI layers of equal thickness over a 401x201 lattice at 5 m (the
    geometry is not printed; this stands in for it), cells of 5x5
    intervals, one surface source, qP and qSV.  CHERT: 1-degree class cache
    (built inside the timed call) and the cached cell network; MSPM:
    chert_trace_mspm, every visited cell's corners solved afresh.  Both
    with the MEV kernel and 1440 sweep samples.  Reports both times, the
    speed-up and the CHERT - MSPM traveltime differences."""
    import torch
    import paper_2609_26108_amd as C
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    cls_np = rock_table_classes()
    K = cls_np.shape[0]
    cls = torch.from_numpy(cls_np).to(dev)
    nx, nz, h, cn = 401, 201, 5.0, 5
    ncx, ncz = (nx - 1) // cn, (nz - 1) // cn
    Z = np.repeat(np.arange(nz)[:, None], nx, 1)
    cid_np = np.minimum(Z * K // nz, K - 1).astype(np.int32).reshape(-1)
    cid = torch.from_numpy(cid_np).to(dev)
    cg = C.make_cell_grid(ncx, ncz, cn, h, h, cid)
    src = [nx // 2 - (nx // 2) % cn]
    n = nx * nz
    node = torch.from_numpy(((np.arange(nx)[None, :] % cn == 0) |
                             (np.arange(nz)[:, None] % cn == 0)).reshape(-1)).to(dev)
    res = {"metric": METRIC, "workload": "mspm", "n_gpus": 1, "dtype": "f64",
           "data": "the paper's rock-property table as four flat VTI layers (synthetic geometry)",
           "config": {"workload": f"CHERT vs MSPM, {ncx}x{ncz} cells of {cn}x{cn} intervals on "
                                  "a 401x201 lattice @5 m, 4 rock-table layers, one surface "
                                  "source, MEV, 1440 sweep samples", "modes": ["qP", "qSV"]}}
    outs = C.OUT_ALL
    per = {}
    for mode, name in ((0, "qP"), (1, "qSV")):
        t = {k: torch.empty((1, n), dtype=dt, device=dev) for k, dt in
             (("tr", torch.float64), ("ti", torch.float64), ("ts", torch.float64),
              ("pp", torch.int32), ("pa", torch.int32))}
        tm = {k: torch.empty_like(v) for k, v in t.items()}
        # CHERT: cache build + cached network
        desc = C.cache_desc(n_dirs=360, modes=(mode,), n_sweep=1440)
        lay = C.chert_cache_layout_of(desc, K)
        cache = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=dev)
        cws = torch.empty(max(C.chert_build_cache_workspace_bytes(desc, K), 1),
                          dtype=torch.uint8, device=dev)
        o = C.trace_opts(outs, bucket_width=16.0)
        tws = torch.empty(C.chert_trace_cells_workspace_bytes(desc, K, cg, 1, o),
                          dtype=torch.uint8, device=dev)

        def chert():
            C.chert_build_cache(desc, cls, K, cache, cws, stream=stream)
            C.chert_trace_cells(desc, cache, K, cg, mode, src, o, t["tr"], t["ti"], t["ts"],
                                t["pp"], t["pa"], tws, stream=stream)
        chert()
        ev = _events(torch, stream)
        for _ in range(max(args.steps, 1)):
            chert()
        t_chert = _elapsed(torch, ev, stream) / max(args.steps, 1)
        # MSPM
        st = C.TraceStats()
        om = C.trace_opts(outs, bucket_width=16.0, stats=st)
        mws = torch.empty(C.chert_trace_mspm_workspace_bytes(K, cg, 1, om), dtype=torch.uint8,
                          device=dev)
        ev = _events(torch, stream)
        C.chert_trace_mspm(cls, K, cg, mode, src, om, tm["tr"], tm["ti"], tm["ts"], tm["pp"],
                           tm["pa"], mws, kernel=C.KERNEL_MEV, n_sweep=1440, stream=stream)
        t_mspm = _elapsed(torch, ev, stream)
        per[name] = {"chert_s": t_chert, "mspm_s": t_mspm, "speedup": t_mspm / t_chert,
                     "mspm_rounds": st.rounds[0], "mspm_cell_visits": st.tile_visits[0],
                     "mspm_corner_solves": st.edge_relaxations[1],
                     "mspm_solves_per_s": st.edge_relaxations[1] / t_mspm,
                     "tauR_chert_minus_mspm": _misfit(t["tr"][0][node], tm["tr"][0][node]),
                     "tauI_chert_minus_mspm": _misfit(t["ti"][0][node], tm["ti"][0][node])}
        print(json.dumps({"progress": name, **{k: v for k, v in per[name].items()
                                               if not isinstance(v, dict)}}), flush=True)
    res["modes"] = per
    # control: rock layer 1 alone (no interfaces, so MSPM's reconstruction
    # is exact): CHERT - MSPM is then the 1-degree binning alone
    cid1 = torch.zeros_like(cid)
    cg1 = C.make_cell_grid(ncx, ncz, cn, h, h, cid1)
    ctrl = {}
    for mode, name in ((0, "qP"), (1, "qSV")):
        desc = C.cache_desc(n_dirs=360, modes=(mode,), n_sweep=1440)
        lay = C.chert_cache_layout_of(desc, 1)
        cache = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=dev)
        cws = torch.empty(max(C.chert_build_cache_workspace_bytes(desc, 1), 1),
                          dtype=torch.uint8, device=dev)
        C.chert_build_cache(desc, cls[:1], 1, cache, cws, stream=stream)
        o = C.trace_opts(C.OUT_TAU_R | C.OUT_TAU_I)
        a_r, a_i, b_r, b_i = (torch.empty((1, n), dtype=torch.float64, device=dev)
                              for _ in range(4))
        tws = torch.empty(C.chert_trace_cells_workspace_bytes(desc, 1, cg1, 1, o),
                          dtype=torch.uint8, device=dev)
        C.chert_trace_cells(desc, cache, 1, cg1, mode, src, o, a_r, a_i, None, None, None, tws,
                            stream=stream)
        mws = torch.empty(C.chert_trace_mspm_workspace_bytes(1, cg1, 1, o), dtype=torch.uint8,
                          device=dev)
        C.chert_trace_mspm(cls[:1], 1, cg1, mode, src, o, b_r, b_i, None, None, None, mws,
                           n_sweep=1440, stream=stream)
        torch.cuda.synchronize()
        ctrl[name] = {"tauR_chert_minus_mspm": _misfit(a_r[0][node], b_r[0][node]),
                      "tauI_chert_minus_mspm": _misfit(a_i[0][node], b_i[0][node])}
    res["uniform_layer1_control"] = ctrl
    res["value"] = float(np.mean([v["speedup"] for v in per.values()]))
    res["unit"] = "x (MSPM time / CHERT time incl. cache build, same network, mean of qP, qSV)"
    res["higher_is_better"] = True
    if not args.no_cpu:
        import oracle as O
        t0 = time.perf_counter()
        O.trace_mspm_2d(ncx, ncz, cn, h, h, cid_np, cls_np, 0, src[0], n_sweep=1440)
        el = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": el, "unit": "s per qP field (oracle MSPM form)",
                               "cores": 1, "kind": "oracle",
                               "sample": "one qP field of the same network; the oracle solves "
                                         "each (class, direction) once, so this is not MSPM's "
                                         "cost"}
    print(json.dumps(res))


def useful_edges_3d(nx, ny, nz, ox, oy, oz):
    return int(sum((nx - abs(a)) * (ny - abs(b)) * (nz - abs(c)) for a, b, c in zip(ox, oy, oz)))


def run_3d(args):
    """3D layered TTI (201 x 201 x 101 at 10 m, 6 classes, qP/qSV): cache on
    41,253 Fibonacci directions, then tau_R and tau_I for four sources and
    both modes in one batch."""
    import torch
    import paper_2609_26108_amd as C
    import workloads as W
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    m = W.config5()
    K = len(m.layers)
    cls = torch.from_numpy(np.stack([C.chert_class_from_thomsen(*L.thomsen_args()).as_array()
                                     for L in m.layers])).to(dev)
    desc = C.cache_desc(dim=3, n_dirs=m.n_dirs, modes=m.modes)
    lay = C.chert_cache_layout_of(desc, K)
    cache = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=dev)
    cws = torch.empty(C.chert_build_cache_workspace_bytes(desc, K), dtype=torch.uint8, device=dev)
    cid = torch.from_numpy(m.class_id.reshape(-1).astype(np.int32)).to(dev)
    grid = C.make_grid3(m.nx, m.ny, m.nz, m.h, m.radius, cid)
    S, n = len(m.sources), m.n_nodes
    stats = C.TraceStats()
    opts = C.trace_opts(C.OUT_TAU_R | C.OUT_TAU_I, stats=stats)
    outs = {mode: (torch.empty((S, n), dtype=torch.float64, device=dev),
                   torch.empty((S, n), dtype=torch.float64, device=dev)) for mode in m.modes}
    b = C.Batch()
    for mode in m.modes:
        b.add(desc, cache, K, grid, mode, m.sources, tau_r=outs[mode][0], tau_i=outs[mode][1])
    tws = torch.empty(C.chert_trace_autotune_workspace_bytes(b, opts), dtype=torch.uint8,
                      device=dev)
    C.chert_build_cache(desc, cls, K, cache, cws, stream=stream)
    t0 = time.perf_counter()
    probe_ms = C.chert_trace_autotune(b, opts, tws, stream=stream)
    tune = {"s": time.perf_counter() - t0, "probe_ms": probe_ms,
            "launch": LAUNCH_NAMES[opts.launch]}
    if opts.launch == C.LAUNCH_FRONTIER:
        tune["bucket_width"] = opts.bucket_width
    else:  # 3D tiles tile_x x tile_x x tile_z
        tune["tile"] = [opts.tile_x, opts.tile_x, opts.tile_z]
        tune["push_group"] = opts.push_group
    ox, oy, oz, _, _ = C.chert_star_3d(m.radius, m.h, m.h, m.h, m.n_dirs)
    E = useful_edges_3d(m.nx, m.ny, m.nz, ox, oy, oz)
    times = {"build": [], "trace": []}
    for rep in range(1 + max(args.steps // 10, 1)):
        ev = _events(torch, stream)
        C.chert_build_cache(desc, cls, K, cache, cws, stream=stream)
        tb = _elapsed(torch, ev, stream)
        ev = _events(torch, stream)
        C.chert_trace_batch(b, opts, tws, stream=stream)
        tt = _elapsed(torch, ev, stream)
        if rep > 0:  # the first pass warms up
            times["build"].append(tb)
            times["trace"].append(tt)
    tb, tt = float(np.mean(times["build"])), float(np.mean(times["trace"]))
    st = C.cache_views(cache, desc, K)[1]
    conv = _converged(st[list(m.modes)].cpu().numpy())
    fields = 2 * len(m.modes) * S
    far = outs[m.modes[0]][0][0, -1].item()
    if not np.isfinite(far):
        raise RuntimeError("3D bench produced an unreachable far corner")
    res = {"metric": METRIC, "workload": "3d", "n_gpus": 1, "dtype": "f64",
           "data": "synthetic (seeded workloads.config5)",
           "config": {"workload": "3D layered TTI 201x201x101 @10 m, 6 classes, qP/qSV, "
                                  "41,253 Fibonacci directions, radius 3 (290 offsets), 4 sources",
                      "nodes": n, "offsets": len(ox), "fields": fields},
           "cache_build_s": tb, "hamiltonian_solves_per_s": conv / tb, "converged_entries": conv,
           "trace_s": tt, "useful_edges_per_field": E,
           "useful_edge_relaxations_per_s": E * fields / tt,
           "raw_over_useful": stats.edge_relaxations[0] / (E * fields),
           "iterations_or_rounds": stats.rounds[0], "repeats": len(times["trace"]),
           "autotune": tune,
           "ms_per_step": 1e3 * (tb + tt)}
    # the surrogate-started 3D build beside the plain one (the MLP is
    # trained once, before it is timed)
    blob, tinfo = train_surrogate(args, dev, stream)
    warm = torch.zeros(lay.total_bytes, dtype=torch.uint8, device=dev)
    wws = torch.empty(C.chert_build_cache_surrogate_workspace_bytes(desc, K), dtype=torch.uint8,
                      device=dev)
    wst = torch.zeros(C.WARM_NSTATS, dtype=torch.int64, device=dev)
    C.chert_build_cache_surrogate(desc, cls, K, blob, warm, wws, wst, stream=stream)  # warm-up
    tw = []
    for _ in range(3):
        ev = _events(torch, stream)
        C.chert_build_cache_surrogate(desc, cls, K, blob, warm, wws, wst, stream=stream)
        tw.append(_elapsed(torch, ev, stream))
    t_warm = float(np.mean(tw))
    fw, sw = C.cache_views(warm, desc, K)
    fp, sp = C.cache_views(cache, desc, K)
    mm = list(m.modes)
    same = bool(torch.equal(sw[mm], sp[mm]))
    okm = (sp[mm] & (1 | 4 | 8)) == 0
    relv = ((fw[0][mm][okm] - fp[0][mm][okm]).abs() / fp[0][mm][okm].abs()).max().item()
    res["warm_start"] = {"training": tinfo, "cache_build_s": t_warm,
                         "hamiltonian_solves_per_s": conv / t_warm,
                         "gain_over_plain": tb / t_warm,
                         "stats": dict(zip(C.WARM_STATS, wst.cpu().numpy().tolist())),
                         "status_equals_plain": same, "V_rel_max_vs_plain": relv}
    res["value"] = res["useful_edge_relaxations_per_s"]
    res["unit"] = "useful edge relaxations/s (3D trace, 16 fields)"
    res["higher_is_better"] = True
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline_3d(m)
    print(json.dumps(res))


def cpu_baseline_3d(m):
    """The CPU oracle as it stands on a bounded sample of the 3D workload:
    its cache build for one class and mode on 200 directions, and its
    Dijkstra for one field on a 41 x 41 x 21 corner of the grid."""
    import oracle as O
    O.build(force=False)
    cls = np.stack([O.class_from_thomsen(*L.thomsen_args()) for L in m.layers])
    t0 = time.perf_counter()
    f, s = O.build_cache_3d(cls[:1], N=200, mode_mask=0b010)
    t1 = time.perf_counter()
    fs, ss = O.build_cache_3d(cls, N=m.n_dirs // 64, mode_mask=0b001, n_sweep=360)
    nx, ny, nz = 41, 41, 21
    sub = np.ascontiguousarray(m.class_id[:nz, :ny, :nx])
    t2 = time.perf_counter()
    O.trace_3d(nx, ny, nz, m.h, m.h, m.h, sub, m.radius, fs[0, 0], fs[1, 0], ss[0], 0,
               N=m.n_dirs // 64)
    t3 = time.perf_counter()
    ox, oy, oz, _, _ = O.star_3d(m.radius, m.h, m.h, m.h, m.n_dirs // 64)
    Es = useful_edges_3d(nx, ny, nz, ox, oy, oz)
    return {"value": Es * 2 / (t3 - t2), "unit": "useful edge relaxations/s (Dijkstra, tau_R + "
                                                 "tau_I of one source)",
            "cores": 1, "kind": "oracle",
            "sample": "Dijkstra on a 41x41x21 corner (2 fields); cache build of 200 directions "
                      "of one class and mode",
            "cache_solves_per_s": 200 / (t1 - t0), "trace_s": t3 - t2,
            "cpu_count": os.cpu_count()}


def cpu_baseline_complex(m, rows, sub, nodes):
    """The CPU oracle as it stands: its plain cache build on a few nodes
    (extrapolated per entry) and its Dijkstra on the full per-node field."""
    import oracle as O
    O.build(force=False)
    cls = np.stack([O.class_from_thomsen(*r) for r in rows[nodes]])
    t0 = time.perf_counter()
    f, s = O.build_cache_2d(cls, mode_mask=1 << m.modes[0], subset=sub)
    t1 = time.perf_counter()
    conv = _converged(s[m.modes[0]])
    return {"value": conv / (t1 - t0), "unit": "converged cache entries/s (plain oracle build)",
            "cores": 1, "kind": "oracle",
            "sample": f"plain cache build of {len(nodes)} solid nodes of the timing sample, "
                      "qSV, star bins",
            "build_s": t1 - t0, "cpu_count": os.cpu_count()}


if __name__ == "__main__":
    main()
