#!/usr/bin/env python3
"""Benchmark: 4-motif counting on an R-MAT graph (scale 20, edge factor 16,
(a,b,c,d) = (0.57, 0.19, 0.19, 0.05)), vertex-induced motifs answered by
pattern morphing (Section 4.2 "Naive PMR": the clique plus the edge-induced
superpatterns are matched, Corollary 3.1 converts back).

One step = submit the six connected vertex-induced 4-vertex patterns, let
the engine plan, match (HIP kernels), copy back and convert, with the graph
resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "motif-count s (morphed vs plain), matches/s, % HBM peak, p50/p99 query latency"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(g, budget_s: float = 15.0):
    """The oracle (tier A injective-map counting of the six vertex-induced
    4-vertex motifs) on a bounded sample of roots of the same graph, on all
    host threads.  Rate = (matches / |Aut|) per second, i.e. matched
    subgraphs credited to the sampled roots."""
    import oracle
    from oracle import P
    pats = list(P.connected_classes(4))
    auts = {m: P.num_automorphisms(4, m) for m in pats}
    deg = g.degrees()
    # a fixed spread of generator ids; roots above degree 256 are left out
    # because one hub root alone costs the oracle d^3 maps
    sample = [r for r in range(0, g.n, 997) if deg[r] <= 256][:4096]
    credited = 0.0
    roots = 0
    t0 = time.perf_counter()
    for r in sample:
        for m in pats:
            credited += oracle.count_maps(g, 4, m, True, roots=(r, r + 1)) / auts[m]
        roots += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {
        "value": credited / dt,
        "unit": "matches/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"tier A vertex-induced 4-motif matching rooted at {roots} vertices "
                  f"(every 997th generator id with degree <= 256), {dt:.1f} s",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--plain-scale", type=int, default=12)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_2012_04553_amd as pm
    from paper_2012_04553_amd.binding import lib

    log(f"generating R-MAT scale {args.scale}")
    t = time.perf_counter()
    g = gen.rmat(args.scale, 16, 0.57, 0.19, 0.19, 0.05, seed=2)
    log(f"  n={g.n} m={g.m} ({time.perf_counter() - t:.1f} s)")

    eng = pm.Engine(arena_bytes=48 << 30)
    t = time.perf_counter()
    gid = eng.load(g)
    load_s = time.perf_counter() - t
    log(f"  loaded in {load_s:.2f} s: {eng.graph_stats(gid)}")

    from oracle import P  # pattern masks only (the six connected 4-vertex classes)
    masks = list(P.connected_classes(4))
    pats = [(4, m, True) for m in masks]

    # untimed pass with the byte tally (same kernel, counting build)
    eng.set_option("count_bytes", 1)
    ref = eng.count(gid, pats, morph=pm.MORPH_NAIVE)
    st = eng.last_stats()
    alg_bytes = st["alg_bytes"]
    launches = st["launches"]
    eng.set_option("count_bytes", 0)
    log(f"  counts {ref}; algorithmic bytes {alg_bytes / 1e9:.2f} GB in {launches} launches")

    for _ in range(args.warmup):
        eng.count(gid, pats, morph=pm.MORPH_NAIVE)

    torch.cuda.synchronize()
    kernel_ms = []
    step_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        out = eng.count(gid, pats, morph=pm.MORPH_NAIVE)
        step_ms.append((time.perf_counter() - ts) * 1e3)
        kernel_ms.append(eng.last_stats()["kernel_ms"])
        assert out == ref, "non-deterministic counts"
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    matches = sum(ref)
    value = matches / (ms_per_step / 1e3)
    k_ms = float(np.mean(kernel_ms))
    achieved = alg_bytes / (k_ms / 1e3) / 1e9

    # morphed vs plain on a graph small enough for plain matching
    mvp = None
    if args.plain_scale > 0:
        gs = gen.rmat(args.plain_scale, 16, seed=2)
        gsid = eng.load(gs)
        res = {}
        for mode, name in ((pm.MORPH_NAIVE, "morphed"), (pm.MORPH_NONE, "plain")):
            eng.count(gsid, pats, morph=mode)
            ts = time.perf_counter()
            c = eng.count(gsid, pats, morph=mode)
            res[name] = (time.perf_counter() - ts, c)
        assert res["morphed"][1] == res["plain"][1], "morphed and plain disagree"
        mvp = {"workload": f"R-MAT scale {args.plain_scale} ef16, 4-motif",
               "morphed_s": round(res["morphed"][0], 4), "plain_s": round(res["plain"][0], 4),
               "speedup": round(res["plain"][0] / res["morphed"][0], 2)}
        eng.graph_unload(gsid)
        log(f"  morphed vs plain: {mvp}")

    cpu = None
    if not args.no_cpu:
        log("  timing the oracle on a bounded sample")
        cpu = cpu_baseline(g)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "matches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": f"4-motif counting (6 vertex-induced motifs, morphed), R-MAT scale {args.scale} "
                        "edge factor 16 (0.57,0.19,0.19,0.05) seed 2",
            "n": g.n, "m": g.m, "motif_count_s": ms_per_step / 1e3,
            "kernel_ms": k_ms, "graph_load_s": round(load_s, 3),
            "matches_per_step": matches,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "match_kernel",
            "launches_per_step": launches,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "alg_bytes_per_step": alg_bytes,
        },
        "morphed_vs_plain": mvp,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    eng.graph_unload(gid)
    eng.close()


if __name__ == "__main__":
    main()
