#!/usr/bin/env python3
"""Throughput benchmark of the plain RPQ path on one MI355X.

Workload (default): R-MAT scale 18 (262,144 vertices, 4,194,304 drawn edges,
8 labels Zipf(1.1), seed 18) with five all-pairs queries, one evaluation each:
a*, a.b*, (a|b).c*, a.b*.c, (a.b)*.  One step evaluates all five from all
262,144 sources to the fixpoint, returning count, checksum and per-source
(count, checksum).  The graph is built (and resident in HBM) before timing;
query compilation, traversal and extraction are inside the timed region.

Metric: product-graph edges per second (sum over sources of the product
edges examined, counted on the Glushkov automaton), with distinct result
pairs per second beside it.

Prints one JSON line.  --gpus > 1 is not supported by this single-GPU build.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat18_l8")
    ap.add_argument("--batch-width", type=int, default=0)
    ap.add_argument("--concurrency", type=int, default=0)
    ap.add_argument("--sync-every", type=int, default=0)
    ap.add_argument("--chunk-edges", type=int, default=0)
    ap.add_argument("--cpu-baseline-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline leg (0 disables it)")
    ap.add_argument("--traffic-file", default=os.path.join(ROOT, "profiles", "expand_rmat18_traffic.json"),
                    help="measured HBM bytes per expand launch (from rocprofv3 --pmc), if present")
    ap.add_argument("--queries", default="",
                    help="comma-separated subset of the workload's queries (profiling runs only)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def copy_calibration(mib):
    """A plain copy of known size: HBM counters of this kernel scale the traversal's counters."""
    import torch
    n = mib << 20
    x = torch.ones(n, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "repeats": 3}), flush=True)


def cpu_baseline(el, queries, budget_s):
    """The oracle as it stands, on the host cores, over a bounded source sample."""
    import numpy as np

    import oracle
    import synth
    threads = max(1, min(os.cpu_count() or 1, 16))
    og = oracle.OracleGraph.from_edgelist(el)
    n = 32
    while True:
        src = synth.sample_sources(el.n_vertices, n, seed=7001)
        t0 = time.perf_counter()
        eprod = 0
        pairs = 0
        for q in queries:
            r = oracle.rpq(og, q, sources=src, pairs=False, threads=threads)
            eprod += r.product_edges
            pairs += r.count
        dt = time.perf_counter() - t0
        if dt >= budget_s / 2 or n >= el.n_vertices or n >= 8192:
            break
        n = min(el.n_vertices, n * 2 if dt * 4 < budget_s else n * 2)
    return dict(value=eprod / dt, unit="product-graph edges/s", cores=threads, kind="oracle",
                pairs_per_s=pairs / dt,
                sample="%d seeded sources (of %d) x %d queries, %.1f s, %d product edges" % (
                    n, el.n_vertices, len(queries), dt, eprod))


def main():
    args = parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU (one MI355X); --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2602_20748_amd as rpq
    import synth

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib)
        return
    rpq.load_library()
    spec = synth.WORKLOADS[args.workload]
    queries = spec["queries"]
    if args.queries:
        queries = [q for q in args.queries.split(",") if q]
    print("bench: generating %s" % args.workload, file=sys.stderr, flush=True)
    el = synth.workload_graph(args.workload)
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    info = g.info()
    opts = dict(batch_width=args.batch_width, concurrency=args.concurrency, sync_every=args.sync_every,
                chunk_edges=args.chunk_edges)
    per_source = torch.zeros((el.n_vertices, 2), dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    qtimes = {q: 0.0 for q in queries}

    def step():
        out = []
        for q in queries:
            t = time.perf_counter()
            nfa = rpq.rpq_nfa_compile(q, el.names)
            out.append(rpq.rpq_eval(g, nfa, None, opts=opts, per_source=per_source))
            qtimes[q] += time.perf_counter() - t
        return out

    for i in range(args.warmup):
        print("bench: warmup %d" % i, file=sys.stderr, flush=True)
        step()
    torch.cuda.synchronize()
    for q in queries:
        qtimes[q] = 0.0
    rpq.rpq_profile_read(reset=True)
    rpq.rpq_profile_enable(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    eprod = 0
    pairs = 0
    per_query = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        res = step()
        for q, r in zip(queries, res):
            eprod += r.product_edges
            pairs += r.count
            per_query[q] = dict(count=r.count, hash="%016x" % r.hash, product_edges=r.product_edges,
                                levels=r.levels, max_depth=r.max_depth)
        print("bench: step %d done" % i, file=sys.stderr, flush=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rpq.rpq_profile_enable(False)
    prof = rpq.rpq_profile_read(reset=True)
    secs = ev0.elapsed_time(ev1) / 1e3
    ms_per_step = secs * 1e3 / args.steps
    for q in queries:
        per_query[q]["ms"] = round(qtimes[q] * 1e3 / max(1, args.steps), 3)

    # roofline of the dominant kernel (level expansion): algorithmic bytes per launch
    # = 4 B per edge item + 16 B per descriptor + 8 B per frontier word read
    #   + 8 B per visited-word read + 16 B per next-word atomic OR (read + write)
    launches = max(1, prof["expand_launches"])
    alg_bytes = (4 * prof["edge_items"] + 16 * prof["descriptors"] + 8 * prof["row_words"]
                 + 8 * prof["word_reads"] + 16 * prof["word_updates"])
    bytes_per_launch = alg_bytes / launches
    avg_ms = prof["expand_ms"] / launches
    achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9 if avg_ms > 0 else 0.0
    traffic = None
    if os.path.exists(args.traffic_file):
        try:
            traffic = json.load(open(args.traffic_file)).get("bytes_per_launch")
        except Exception:
            traffic = None
    roofline = dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBPS, 5), traffic=traffic,
                    kernel="k_expand", avg_launch_ms=round(avg_ms, 5), launches=prof["expand_launches"],
                    alg_bytes_per_launch=round(bytes_per_launch, 1),
                    expand_share=round(prof["expand_ms"] / max(1e-9, prof["expand_ms"] + prof["finalize_ms"]), 4),
                    finalize_avg_ms=round(prof["finalize_ms"] / max(1, prof["finalize_launches"]), 5),
                    counters={k: prof[k] for k in ("edge_items", "descriptors", "row_words", "word_reads",
                                                   "word_updates", "expand_ms", "finalize_ms")})
    cpu = None
    if args.cpu_baseline_seconds > 0:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(el, queries, args.cpu_baseline_seconds)
    line = {
        "metric": "product-graph edges/sec",
        "value": eprod / secs,
        "unit": "product-graph edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (seeded R-MAT; no dataset)",
        "config": {"workload": "%s: R-MAT scale 18, %d vertices, %d drawn / %d distinct edges, %d labels Zipf(1.1);"
                               " all-pairs %s; plain form, one evaluation per query"
                               % (args.workload, el.n_vertices, el.n_edges, info["n_edges"], el.n_labels,
                                  ", ".join(queries)),
                   "sources": el.n_vertices, "queries": queries, "form": "plain",
                   "opts": {k: v for k, v in opts.items() if v}},
        "distinct_pairs_per_s": pairs / secs,
        "wall_s": wall,
        "per_query": per_query,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    g.close()


if __name__ == "__main__":
    main()
