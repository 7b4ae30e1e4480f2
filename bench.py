#!/usr/bin/env python3
"""Benchmark of the pattern-morphing engine on one MI355X.

Default workload: 4-motif counting on an R-MAT graph (scale 20, edge factor
16, (a,b,c,d) = (0.57, 0.19, 0.19, 0.05), seed 2).  The six vertex-induced
4-vertex motifs are answered by pattern morphing (Section 4.2, Naive PMR:
the clique plus the edge-induced superpatterns are matched, Corollary 3.1
converts back).  One step = submit the six patterns, plan, match (one
hipGraph replay of the persistent multi-pattern launches), copy back and
convert, with the graph resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1]
    python bench.py --workload {rmat20-4mc,er2000-4mc,rmat-5mc,rmat18-fsm,serving}

The other workloads print a line of the same form for the other
configurations (plain ER 4-motif counting, batched 5-motif counting at a
reduced scale, labeled 3-edge FSM with MNI support, and the serving loop).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "motif-count s (morphed vs plain), matches/s, % HBM peak, p50/p99 query latency"
# sources that decide the match kernel's memory traffic (kernel, plans, launch configuration)
PATH_SRCS = [os.path.join(ROOT, "paper_2012_04553_amd", "csrc", f)
             for f in ("kernels.hip", "kernels.hpp", "planner.cpp", "runtime.hpp", "runtime.cpp")]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def path_sha():
    h = hashlib.sha256()
    for p in PATH_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed PMC summary
    (profiles/<kernel>_rmat20_4mc_traffic.md), or None when a kernel, the
    planner or the launch set-up changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_rmat20_4mc_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            w = line.strip().split()
            if len(w) == 2 and w[0].endswith(":"):
                vals[w[0][:-1]] = w[1]
    if vals.get("path_source_sha256") != path_sha():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def base_line(args, value, unit, ms_per_step, workload, extra_cfg, higher=True):
    return {
        "metric": METRIC,
        "value": value,
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": higher,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": dict({"workload": workload}, **extra_cfg),
    }


def timed_steps(eng, step, args):
    """W untimed steps, then K timed ones bracketed by device syncs."""
    import torch
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        kms.append(eng.last_stats()["kernel_ms"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall * 1e3 / args.steps, kms


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_4mc(g, stride: int = 2, graph_desc: str = "R-MAT scale-20 graph", min_s: float = 0.0):
    """The oracle's tier-C computation of the same six counts (closed forms
    over degrees and per-edge common neighbours, 4-cycles by co-degrees,
    4-cliques on the degree DAG; vertex-induced counts by Corollary 3.1) on
    a bounded sample of the same graph: the roots u with u % stride == 0,
    each credited with exactly its share of every sum, on all host
    threads.  Rate = vertex-induced subgraphs credited to the sample per
    second (Corollary 3.1 is linear, so credited shares convert like
    totals).  A small graph is timed over repeated passes, min_s at least."""
    import numpy as np
    import oracle
    from oracle import P
    t0 = time.perf_counter()
    reps = 0
    while True:
        raw = oracle.tier_c4_sample(g, stride, 0)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= min_s:
            break
    # credited edge-induced shares (the divisions of the full closed forms)
    ei = {"star3": raw["star3"], "path4": raw["path4"] - raw["triangles"],
          "tailed_triangle": raw["tailed_triangle"], "cycle4": raw["cycle4"] / 2,
          "diamond": raw["diamond"], "clique4": raw["clique4"]}
    names = oracle.named_4()
    cls, mat = P.morph_matrix(4)
    ne = np.array([float(ei[k]) for k in (next(n for n in names if names[n] == m) for m in cls)])
    nv = np.linalg.solve(np.array(mat, dtype=np.float64), ne)
    credited = float(nv.sum())
    roots = (g.n + stride - 1) // stride
    which = f"every {stride}th root ({roots} of {g.n})" if stride > 1 else f"all {g.n} roots"
    return {
        "value": credited * reps / dt,
        "unit": "matches/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"tier-C closed forms of the six 4-vertex counts (Corollary 3.1 for the vertex-induced ones) "
                  f"credited to {which} of the same {graph_desc}, {reps} pass(es) in "
                  f"{dt:.1f} s on {oracle.num_threads()} threads of {cpu_model()}",
        "seconds": round(dt, 2),
        "cpu_model": cpu_model(),
    }


def launch_roofline(eng, gid, pats, mode, steps):
    """Per-launch roofline: algorithmic bytes of every launch (byte-counting
    build, untimed) and its device time between HIP events on the engine's
    stream, averaged over `steps` eager passes of the same launch set."""
    eng.set_option("count_bytes", 1)
    eng.count(gid, pats, morph=mode)
    bytes_ = [x["alg_bytes"] for x in eng.launch_stats()]
    names = [x["kernel"] for x in eng.launch_stats()]
    eng.set_option("count_bytes", 0)
    log("  per-launch bytes done")
    eng.set_option("launch_events", 1)
    ms = [0.0] * len(bytes_)
    eng.count(gid, pats, morph=mode)
    log("  per-launch timing warm-up done")
    for _ in range(steps):
        eng.count(gid, pats, morph=mode)
        for i, x in enumerate(eng.launch_stats()):
            ms[i] += x["ms"] / steps
        log("  per-launch timing pass done")
    eng.set_option("launch_events", 0)
    per = []
    for name, b, t in zip(names, bytes_, ms):
        per.append({"kernel": name, "alg_bytes": b, "ms": round(t, 4),
                    "gbs": round(b / (t / 1e3) / 1e9, 1) if t > 0 else None})
    return per


# ---------------------------------------------------------------- workloads

def run_4mc(args, eng, g, workload, morph_name="morphed"):
    import paper_2012_04553_amd as pm
    import gen
    masks = list(gen.connected_masks(4))
    pats = [(4, m, True) for m in masks]
    mode = pm.MORPH_NAIVE if morph_name == "morphed" else pm.MORPH_NONE
    t = time.perf_counter()
    gid = eng.load(g)
    load_s = time.perf_counter() - t
    log(f"  loaded in {load_s:.2f} s: {eng.graph_stats(gid)}")
    # untimed pass with the byte tally (same kernel, counting build)
    eng.set_option("count_bytes", 1)
    ref = eng.count(gid, pats, morph=mode)
    st = eng.last_stats()
    alg_bytes = st["alg_bytes"]
    launches = st["launches"]
    eng.set_option("count_bytes", 0)
    log(f"  counts {ref}; algorithmic bytes {alg_bytes / 1e9:.2f} GB in {launches} launches")

    def step():
        out = eng.count(gid, pats, morph=mode)
        assert out == ref, "non-deterministic counts"

    ms_per_step, kms = timed_steps(eng, step, args)
    matches = sum(ref)
    k_ms = sum(kms) / len(kms)
    per_launch_ms = k_ms / launches
    achieved = (alg_bytes / launches) / (per_launch_ms / 1e3) / 1e9
    line = base_line(args, matches / (ms_per_step / 1e3), "matches/s", ms_per_step, workload, {
        "n": g.n, "m": g.m, "motif_count_s": ms_per_step / 1e3, "kernel_ms": k_ms,
        "graph_load_s": round(load_s, 3), "matches_per_step": matches, "counts": ref,
    })
    per = launch_roofline(eng, gid, pats, mode, max(1, args.steps // 2))
    dom = max(range(len(per)), key=lambda i: per[i]["ms"])
    d = per[dom]
    d_ach = d["alg_bytes"] / (d["ms"] / 1e3) / 1e9 if d["ms"] > 0 else 0.0
    line["roofline"] = {
        "bound": "hbm", "kernel": d["kernel"], "launch_index": dom,
        "achieved": d_ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": d_ach / HBM_PEAK_GBS,
        "traffic": None, "alg_bytes_per_launch": d["alg_bytes"], "avg_launch_ms": d["ms"],
        "all_launches": {"launches_per_step": launches, "alg_bytes_per_step": alg_bytes,
                         "achieved": achieved, "frac": achieved / HBM_PEAK_GBS},
        "per_launch": per,
    }
    return line, gid


def wl_rmat20_4mc(args, eng):
    import gen
    import paper_2012_04553_amd as pm
    log(f"generating R-MAT scale {args.scale}")
    g = gen.rmat(args.scale, 16, 0.57, 0.19, 0.19, 0.05, seed=2)
    log(f"  n={g.n} m={g.m}")
    line, gid = run_4mc(args, eng, g, f"4-motif counting (6 vertex-induced motifs, morphed), R-MAT scale "
                        f"{args.scale} edge factor 16 (0.57,0.19,0.19,0.05) seed 2")
    if args.scale == 20:
        line["roofline"]["traffic"] = measured_traffic(line["roofline"]["kernel"])
    eng.graph_unload(gid)
    # morphed vs plain on a graph small enough for plain matching
    if args.plain_scale > 0:
        gs = gen.rmat(args.plain_scale, 16, seed=2)
        gsid = eng.load(gs)
        pats = [(4, m, True) for m in gen.connected_masks(4)]
        res = {}
        for mode, name in ((pm.MORPH_NAIVE, "morphed"), (pm.MORPH_NONE, "plain")):
            eng.count(gsid, pats, morph=mode)
            ts = time.perf_counter()
            c = eng.count(gsid, pats, morph=mode)
            res[name] = (time.perf_counter() - ts, c)
        assert res["morphed"][1] == res["plain"][1], "morphed and plain disagree"
        line["morphed_vs_plain"] = {
            "workload": f"R-MAT scale {args.plain_scale} ef16, 4-motif",
            "morphed_s": round(res["morphed"][0], 4), "plain_s": round(res["plain"][0], 4),
            "speedup": round(res["plain"][0] / res["morphed"][0], 2)}
        eng.graph_unload(gsid)
        log(f"  morphed vs plain: {line['morphed_vs_plain']}")
    if not args.no_cpu:
        log("  timing the oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline_4mc(g)
    else:
        line["cpu_baseline"] = None
    return line


def wl_er2000_4mc(args, eng):
    import gen
    g = gen.erdos_renyi(2000, 0.005, 1)
    res = {}
    for name in ("plain", "morphed"):
        line, gid = run_4mc(args, eng, g, f"plain 4-motif counting, ER G(2000, 0.005) seed 1 ({name})",
                            morph_name=name)
        eng.graph_unload(gid)
        res[name] = line
    line = res["morphed"]
    line["morphed_vs_plain"] = {"morphed_s": res["morphed"]["ms_per_step"] / 1e3,
                                "plain_s": res["plain"]["ms_per_step"] / 1e3}
    line["config"]["workload"] = "4-motif counting, ER G(2000, 0.005) seed 1, morphed (plain beside it)"
    line["cpu_baseline"] = None if args.no_cpu else cpu_baseline_4mc(g, stride=1, graph_desc="ER(2000, 0.005) graph",
                                                                      min_s=2.0)
    return line


def wl_rmat_5mc(args, eng):
    import gen
    import paper_2012_04553_amd as pm
    scale = args.scale if args.scale != 20 else 10
    g = gen.rmat(scale, 16, 0.57, 0.19, 0.19, 0.05, seed=3)
    gid = eng.load(g)
    pats = [(5, m, True) for m in gen.connected_masks(5)]
    tune = None
    if args.autotune_5mc:
        log(f"  R-MAT scale {scale}: n={g.n} m={g.m}; autotuning the 5-motif closure")
        t = time.perf_counter()
        tune = eng.autotune(gid, pats, morph=pm.MORPH_NAIVE)
        log(f"  autotune {tune} in {time.perf_counter() - t:.1f} s")
    else:
        log(f"  R-MAT scale {scale}: n={g.n} m={g.m}; the engine's default launch configuration")
    eng.set_option("count_bytes", 1)
    t = time.perf_counter()
    ref = eng.count(gid, pats, morph=pm.MORPH_NAIVE)
    st = eng.last_stats()
    eng.set_option("count_bytes", 0)
    log(f"  byte-tally pass in {time.perf_counter() - t:.1f} s")

    def step():
        assert eng.count(gid, pats, morph=pm.MORPH_NAIVE) == ref
        log("  step done")

    ms_per_step, kms = timed_steps(eng, step, args)
    k_ms = sum(kms) / len(kms)
    launches = st["launches"]
    achieved = (st["alg_bytes"] / launches) / (k_ms / launches / 1e3) / 1e9
    line = base_line(args, sum(ref) / (ms_per_step / 1e3), "matches/s", ms_per_step,
                     f"batched 5-motif counting (21 vertex-induced motifs, morphed, "
                     f"{'autotuned' if tune else 'default launch configuration'}, hipGraph), "
                     f"R-MAT scale {scale} edge factor 16 seed 3",
                     {"n": g.n, "m": g.m, "kernel_ms": k_ms, "autotune": tune, "counts": ref,
                      "num_alt": st["num_alt"]})
    per = launch_roofline(eng, gid, pats, pm.MORPH_NAIVE, max(1, args.steps // 2))
    dom = max(range(len(per)), key=lambda i: per[i]["ms"])
    d = per[dom]
    d_ach = d["alg_bytes"] / (d["ms"] / 1e3) / 1e9 if d["ms"] > 0 else 0.0
    line["roofline"] = {"bound": "hbm", "kernel": d["kernel"], "launch_index": dom, "achieved": d_ach,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": d_ach / HBM_PEAK_GBS, "traffic": None,
                        "alg_bytes_per_launch": d["alg_bytes"], "avg_launch_ms": d["ms"],
                        "all_launches": {"launches_per_step": launches, "achieved": achieved,
                                         "frac": achieved / HBM_PEAK_GBS},
                        "per_launch": per}
    line["cpu_baseline"] = None
    eng.graph_unload(gid)
    if args.plain_5mc_scale > 0:
        gp = gen.rmat(args.plain_5mc_scale, 16, 0.57, 0.19, 0.19, 0.05, seed=3)
        gpid = eng.load(gp)
        res = {}
        for mode, name in ((pm.MORPH_NAIVE, "morphed"), (pm.MORPH_NONE, "plain")):
            eng.count(gpid, pats, morph=mode)
            ts = time.perf_counter()
            c = eng.count(gpid, pats, morph=mode)
            res[name] = (time.perf_counter() - ts, c)
        assert res["morphed"][1] == res["plain"][1], "morphed and plain disagree"
        line["morphed_vs_plain"] = {
            "workload": f"R-MAT scale {args.plain_5mc_scale} ef16 seed 3, 21 vertex-induced 5-motifs",
            "morphed_s": round(res["morphed"][0], 4), "plain_s": round(res["plain"][0], 4),
            "speedup": round(res["plain"][0] / res["morphed"][0], 2)}
        eng.graph_unload(gpid)
    return line


def wl_rmat18_fsm(args, eng):
    import gen
    import numpy as np
    import paper_2012_04553_amd as pm
    g = gen.rmat(18, 8, 0.57, 0.19, 0.19, 0.05, seed=4).with_labels(gen.zipf_labels(1 << 18, 16, 1.2, 40))
    gid = eng.load(g)
    # the number of edge-induced 3-edge matches (triangles + 3-paths + 3-stars)
    tri, p4, s3 = [m for m in gen.connected_masks(3) if bin(m).count("1") == 3] + \
        [m for m in gen.connected_masks(4) if bin(m).count("1") == 3]
    c3 = eng.count(gid, [(3, tri, False)], morph=pm.MORPH_NONE)[0]
    c4 = eng.count(gid, [(4, p4, False), (4, s3, False)], morph=pm.MORPH_NONE)
    matches = c3 + sum(c4)
    ref = eng.fsm(gid, 16, 1000)

    per_step = []

    def step():
        sup, freq = eng.fsm(gid, 16, 1000)
        assert np.array_equal(sup, ref[0])
        per_step.append(eng.launch_stats())

    ms_per_step, kms = timed_steps(eng, step, args)
    # per-kernel device time between HIP events on the engine's stream,
    # averaged over the timed steps; algorithmic bytes from the graph's sizes
    timed = per_step[args.warmup:]
    per = []
    for i, x in enumerate(timed[0]):
        ms = sum(t[i]["ms"] for t in timed) / len(timed)
        per.append({"kernel": x["kernel"], "alg_bytes": x["alg_bytes"], "ms": round(ms, 4),
                    "gbs": round(x["alg_bytes"] / (ms / 1e3) / 1e9, 1) if ms > 0 else None})
    dom = max(range(len(per)), key=lambda i: per[i]["ms"])
    d = per[dom]
    d_ach = d["alg_bytes"] / (d["ms"] / 1e3) / 1e9 if d["ms"] > 0 else 0.0
    line = base_line(args, matches / (ms_per_step / 1e3), "matches/s", ms_per_step,
                     "labeled 3-edge FSM, MNI support of all 46,768 labeled patterns, threshold 1000, "
                     "R-MAT scale 18 edge factor 8 seed 4, Zipf(1.2) labels over 16 (seed 40)",
                     {"n": g.n, "m": g.m, "kernel_ms": sum(kms) / len(kms),
                      "frequent": int(ref[1].sum()), "edge_induced_matches": matches})
    line["roofline"] = {"bound": "hbm", "kernel": d["kernel"], "launch_index": dom, "achieved": d_ach,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": d_ach / HBM_PEAK_GBS, "traffic": None,
                        "alg_bytes_per_launch": d["alg_bytes"], "avg_launch_ms": d["ms"], "per_launch": per}
    line["cpu_baseline"] = None
    eng.graph_unload(gid)
    return line


def service_profile(eng, ids, sizes, ks, per_class, deadline_s):
    """Where serving time goes: `per_class` queries of every (graph, k) class
    of the same query distribution, each served alone (one slot, batches of
    one), with their planning and launch-set set-up time and their service
    time (admission to completion).  A query still running at the deadline is
    cancelled and counted as taking the deadline, so the mix estimate below is
    an upper bound on the queries per second one GPU sustains."""
    import gen
    import paper_2012_04553_amd as pm
    pool = gen.query_stream(400 * len(ids) * len(ks) * max(1, per_class), 1e6, len(ids), seed=57,
                            k_choices=ks)
    classes = []
    for gi, gid in enumerate(ids):
        for k in ks:
            qs = [q for q in pool if q.graph == gi and q.patterns[0][0] == k][:per_class]
            reqs = [(0.0, gid, q.patterns, pm.MORPH_COST) for q in qs]
            res, _ = eng.serve(reqs, max_slots=1, max_batch=1, deadline_s=deadline_s, progress_every=1)
            svc = sorted(r["service_s"] if r["status"] == 0 else max(r["service_s"], deadline_s) for r in res)
            setup = [r["setup_s"] for r in res]
            done = sum(1 for r in res if r["status"] == 0)
            row = {"graph_n": sizes[gi], "k": k, "queries": len(res), "completed": done,
                   "timeouts": sum(1 for r in res if r["status"] == -7),
                   "median_service_s": svc[len(svc) // 2] if svc else None,
                   "mean_service_s": sum(svc) / len(svc) if svc else None,
                   "max_service_s": svc[-1] if svc else None,
                   "mean_setup_s": sum(setup) / len(setup) if setup else None}
            log(f"  service profile n={sizes[gi]} k={k}: {row}")
            classes.append(row)
    means = [c["mean_service_s"] for c in classes if c["mean_service_s"] is not None]
    mix = sum(means) / len(means) if means else None
    return {"per_class": per_class, "deadline_s": deadline_s, "classes": classes,
            "mix_mean_service_s": mix, "mix_qps_upper_bound": (1.0 / mix) if mix else None}


def wl_serving(args, eng):
    import gen
    import numpy as np
    import paper_2012_04553_amd as pm
    div = args.serve_div
    sizes = [100000 // div, 500000 // div, 1000000 // div, 4000000 // div]
    ids = []
    for i, n in enumerate(sizes):
        g = gen.chung_lu(n, 2.1, 20.0, seed=51 + i).with_labels(gen.zipf_labels(n, 16, 1.2, 55))
        ids.append(eng.load(g))
        log(f"  Chung-Lu n={n}: m={g.m}")
    ks = tuple(int(x) for x in args.serve_k.split(","))
    profile = service_profile(eng, ids, sizes, ks, args.serve_profile, args.serve_deadline) \
        if args.serve_profile > 0 else None
    qs = gen.query_stream(args.serve_queries, args.serve_qps, 4, seed=56, k_choices=ks)
    reqs = [(q.arrival_s, ids[q.graph], q.patterns, pm.MORPH_COST) for q in qs]
    t = time.perf_counter()
    res, st = eng.serve(reqs, max_slots=8, max_batch=8, budget_bytes=32 << 30, deadline_s=args.serve_deadline,
                        progress_every=max(1, args.serve_queries // 20))
    wall = time.perf_counter() - t
    # outcome per (graph, largest pattern size) class: completed, timed out
    # on the device, shed at admission (a timeout with no service time)
    by_class = {}
    for q, r in zip(qs, res):
        key = f"n={sizes[q.graph]} k={max(p[0] for p in q.patterns)}"
        c = by_class.setdefault(key, {"offered": 0, "completed": 0, "timed_out": 0, "shed": 0, "other": 0})
        c["offered"] += 1
        if r["status"] == 0:
            c["completed"] += 1
        elif r["status"] == -7:
            c["shed" if r["service_s"] == 0.0 else "timed_out"] += 1
        else:
            c["other"] += 1
    line = base_line(args, st["p99_s"], "s (p99 latency)", wall * 1e3,
                     f"serving {args.serve_queries} queries at {args.serve_qps} QPS over 4 Chung-Lu graphs "
                     f"(beta 2.1, mean degree 20, n = {sizes}), k in {ks}, 30% labeled, cost-based morphing",
                     {"p50_s": st["p50_s"], "p99_s": st["p99_s"], "matches_per_s": st["matches_per_s"],
                      "completed": st["completed"], "timeouts": st["timeouts"], "shed": st["shed"],
                      "mean_inflight": st["mean_inflight"], "batches": st["batches"],
                      "sustained_qps": st["sustained_qps"], "offered_qps": args.serve_qps,
                      "mean_setup_s": st["mean_setup_s"], "mean_service_s": st["mean_service_s"],
                      "makespan_s": st["makespan_s"], "deadline_s": args.serve_deadline,
                      "by_class": dict(sorted(by_class.items())), "service_profile": profile}, higher=False)
    line["roofline"] = None
    line["cpu_baseline"] = None
    return line


WORKLOADS = {
    "rmat20-4mc": wl_rmat20_4mc,
    "er2000-4mc": wl_er2000_4mc,
    "rmat-5mc": wl_rmat_5mc,
    "rmat18-fsm": wl_rmat18_fsm,
    "serving": wl_serving,
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat20-4mc", choices=sorted(WORKLOADS))
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--plain-scale", type=int, default=12)
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="after the workload, copy this many MiB device to device once (PMC calibration)")
    ap.add_argument("--plain-5mc-scale", type=int, default=9,
                    help="rmat-5mc: also time plain (unmorphed) 5-motif counting at this scale (0: skip)")
    ap.add_argument("--serve-div", type=int, default=10)
    ap.add_argument("--serve-queries", type=int, default=1000)
    ap.add_argument("--serve-qps", type=float, default=200.0)
    ap.add_argument("--serve-k", default="3,4")
    ap.add_argument("--serve-deadline", type=float, default=0.0)
    ap.add_argument("--autotune-5mc", type=int, default=1,
                    help="rmat-5mc: autotune the launch configuration first (0 = engine defaults)")
    ap.add_argument("--serve-profile", type=int, default=0,
                    help="serving: time this many queries of every (graph, k) class alone first")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(several GPUs would each take a share of the work items and add their counters)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2012_04553_amd as pm

    eng = pm.Engine(arena_bytes=48 << 30)
    line = WORKLOADS[args.workload](args, eng)
    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"  calibration copy of {nbytes} bytes done")
    print(json.dumps(line), flush=True)
    eng.close()


if __name__ == "__main__":
    main()
