"""CHERT hot-path benchmark on one MI355X.

Workload: the 5-layer TTI model (401 x 201 nodes at 5 m, 5 cache classes,
qP/qSV/qSH, 1-degree cache, forward-star radius 5, one surface source),
seeded synthetic parameters (workloads.config2).  One step = the whole hot
path: build the directional cache for all classes and modes
(chert_build_cache), then trace propagation and attenuation traveltimes,
predecessors and t* for every mode in one batched call (chert_trace_batch).  Inputs (classes,
class map) are resident in HBM before the timed region.

Prints one JSON line.  `value` is useful (Dijkstra-equivalent) edge
relaxations per second of whole-step wall time; the breakdown carries
Hamiltonian solves/s of the cache build and shots/s.  The CPU oracle is timed
on the same workload (one step, single thread) as `cpu_baseline`.
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
FP64_PEAK_TFLOPS = 78.6


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
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(shots and cache entries would shard across GPUs with no communication).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2609_26108_amd as C
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
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
    opts = C.trace_opts(C.OUT_ALL)
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
    tws = torch.empty(C.chert_trace_batch_workspace_bytes(batch, opts), dtype=torch.uint8,
                      device=dev)
    stream = torch.cuda.current_stream()

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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(timed=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = 1e3 * wall / args.steps

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
        },
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
    return {"value": E * fields_per_step / (t2 - t0),
            "unit": "useful edge relaxations/s (whole step: cache build + 6 fields)",
            "cores": 1, "kind": "oracle",
            "sample": "one full step of the same workload (cache build + Dijkstra for 3 modes)",
            "build_s": t1 - t0, "trace_s": t2 - t1, "cpu_count": os.cpu_count()}


if __name__ == "__main__":
    main()
