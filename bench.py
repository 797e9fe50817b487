#!/usr/bin/env python3
"""Throughput benchmark of the RPQ hot path on one MI355X.

Default workload: R-MAT scale 23 (8,388,608 vertices, 134,217,728 drawn edges,
16 labels Zipf(1.1), seed 23), the largest graph.  One step evaluates the five
Table 2 query shapes a*, a.b*, (a|b).c*, a.b*.c and (a.b)* to the fixpoint
from a seeded sample of 65,536 sources (all pairs would take hours per step),
with count, checksum and per-source (count, checksum).  The graph is built,
and resident in HBM, before timing.

Legs of the default line:
  plain    one rpq_eval per query (query compile, traversal, extraction); its
           K timed steps give `value` (product-graph edges per second) and the
           roofline of the level expansion, the dominant kernel;
  batched  256 single-source queries (generated regexes) in one persistent,
           graph-captured launch against the same queries as plain launches;
  serving  a short serving run on the same resident graph: a burst (capacity)
           and one Poisson rate of the mixed request stream, p50/p99 latency,
           served edges/s against the same requests run one at a time.
--workload rmat18_l8 gives the all-pairs R-MAT 18 step instead (plain and
batched forms of the five queries plus the batched-vs-plain mixes).
--mix times the 256-query batch on R-MAT scale 22 (autotuned) against its
plain launches; --serve runs the full serving sweep; --crpq times the CRPQs on
the full typed social graph (each prints one JSON line of its own).

Metric: product-graph edges per second (per source, the product edges
examined, counted on the Glushkov automaton), with distinct pairs per second.
--gpus above 1 is refused: the benchmark runs on one GPU.
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


def describe_graph(spec):
    if spec["kind"] == "rmat":
        return "R-MAT scale %d" % spec["scale"]
    return spec["kind"]


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat23_l16")
    ap.add_argument("--form", choices=["batched", "plain"], default="plain",
                    help="which form's throughput is `value` (both are measured)")
    ap.add_argument("--batch-width", type=int, default=0, help="plain form: unit width (0 = default policy)")
    ap.add_argument("--concurrency", type=int, default=0)
    ap.add_argument("--sync-every", type=int, default=0)
    ap.add_argument("--chunk-edges", type=int, default=0)
    ap.add_argument("--visit", choices=["auto", "two-reads", "seen-or"], default="auto",
                    help="plain form: how the expansion finds new bits (auto: by graph size)")
    ap.add_argument("--no-autotune", action="store_true", help="batched form: keep the default plan")
    ap.add_argument("--batched-plan", default="",
                    help="batched form: WIDTH:CHUNK, a fixed plan instead of the autotuner's (profiling runs)")
    ap.add_argument("--cpu-baseline-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline leg (0 disables it)")
    ap.add_argument("--traffic-file", default="",
                    help="measured HBM bytes per launch of the dominant kernels (rocprofv3 --pmc), if present")
    ap.add_argument("--sources", type=int, default=-1,
                    help="plain/batched forms: evaluate from this many seeded sampled sources (0 = all pairs; "
                         "default: the workload's sample size, all pairs where it has none)")
    ap.add_argument("--queries", default="",
                    help="comma-separated subset of the workload's queries (profiling runs only)")
    ap.add_argument("--only", choices=["", "plain", "batched"], default="",
                    help="time only one form (profiling runs only)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (counter calibration)")
    ap.add_argument("--no-mixes", action="store_true",
                    help="skip the batched-vs-plain comparison on many-query mixes")
    ap.add_argument("--mix", action="store_true",
                    help="the 256-query batch on R-MAT scale 22 (generated regexes, half single-source, half "
                         "4,096-source slices): autotuned batched run vs the plain launches")
    ap.add_argument("--plans", action="store_true",
                    help="split plans (loop-cache, start-in-the-middle) of a.b.c* against the one-automaton plan, "
                         "from --sources sampled sources of --workload")
    ap.add_argument("--no-serve-leg", action="store_true", help="skip the serving leg of the default line")
    ap.add_argument("--serve-leg", default="burst,10",
                    help="serving leg of the default line: arrival rates ('burst' = all at once)")
    ap.add_argument("--serve-leg-burst", type=int, default=64, help="serving leg: requests in the burst")
    ap.add_argument("--serve-leg-seconds", type=float, default=8.0, help="serving leg: seconds per rate")
    ap.add_argument("--crpq", action="store_true",
                    help="time the two CRPQs on the full typed social graph (1M persons, 10M messages, 16,384 tags)")
    ap.add_argument("--serve", action="store_true",
                    help="serving measurement instead of the throughput step: Poisson streams of mixed "
                         "requests at each --qps rate (prints one JSON line of its own)")
    ap.add_argument("--qps", default="burst,10,50,100",
                    help="serving: comma-separated arrival rates; 'burst' = every request at once (capacity)")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="serving: measured seconds per rate")
    ap.add_argument("--serve-warmup-seconds", type=float, default=2.0, help="serving: warm-up seconds per rate")
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--serve-resident-slots", type=int, default=8,
                    help="serving: slots of the resident engine that runs the single-source RPQs (0 = off: "
                         "they run on the workers with the hash-set search)")
    ap.add_argument("--serve-resident-iters", type=int, default=8,
                    help="serving: iterations per launch of the resident engine")
    ap.add_argument("--serve-pool-gib", type=float, default=96.0)
    ap.add_argument("--serve-max-requests", type=int, default=4000,
                    help="serving: cap on requests per rate (keeps the FIFO comparison bounded)")
    return ap.parse_args()


def crpq_main():
    """The information-propagation CRPQ (m -hasTag-> t, m -hasCreator-> u, m -replyOf*-> p, t the most
    frequent tag) and the 3-cycle of knows.knows* over seeded person samples, on the full typed social
    graph; wall time of one call after a warm-up call, graph resident."""
    import numpy as np
    import torch

    import paper_2602_20748_amd as rpq
    import synth

    print("bench: generating the social graph", file=sys.stderr, flush=True)
    el = synth.workload_graph("social_p1m_m10m_t16k")
    t = time.perf_counter()
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, vertex_label=el.vertex_label,
                             flags=rpq.RPQ_BUILD_IN_CSR, names=el.names)
    torch.cuda.synchronize()
    ingest_ms = (time.perf_counter() - t) * 1e3
    n_person, n_msg = 1_000_000, 10_000_000
    q1 = [(0, "hasTag", 1), (0, "hasCreator", 2), (0, "replyOf*", 3)]
    kw = dict(binding=[None, n_person + n_msg, None, None], vertex_label=[1, 2, 0, 1])
    cyc = [(0, "knows.knows*", 1), (1, "knows.knows*", 2), (2, "knows.knows*", 0)]
    rng = np.random.default_rng(4004)
    s128 = np.sort(rng.choice(n_person, size=128, replace=False)).astype(np.uint32)
    s1024 = np.sort(rng.choice(n_person, size=1024, replace=False)).astype(np.uint32)
    cases = [("information propagation, count + checksum", lambda: rpq.crpq_eval(g, q1, 4, **kw)),
             ("information propagation, sorted tuples",
              lambda: rpq.crpq_eval(g, q1, 4, tuples=True, capacity=1 << 24, **kw)),
             ("3-cycle of knows.knows*, 128 persons, sorted tuples",
              lambda: rpq.crpq_eval(g, cyc, 3, domain=[s128] * 3, vertex_label=[0] * 3, tuples=True)),
             ("3-cycle of knows.knows*, 1,024 persons, count + checksum",
              lambda: rpq.crpq_eval(g, cyc, 3, domain=[s1024] * 3, vertex_label=[0] * 3)),
             ("3-cycle, 128 persons, sorted tuples, atoms in the batched form",
              lambda: rpq.crpq_eval(g, cyc, 3, domain=[s128] * 3, vertex_label=[0] * 3, tuples=True,
                                    flags=rpq.CRPQ_BATCH_ATOMS)),
             ("3-cycle, 1,024 persons, count + checksum, atoms in the batched form",
              lambda: rpq.crpq_eval(g, cyc, 3, domain=[s1024] * 3, vertex_label=[0] * 3, flags=rpq.CRPQ_BATCH_ATOMS))]
    out = []
    for name, f in cases:
        print("bench: crpq %s" % name, file=sys.stderr, flush=True)
        f()   # warm-up: sizes the workspace
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = f()
        torch.cuda.synchronize()
        out.append(dict(case=name, ms=round((time.perf_counter() - t) * 1e3, 2), count=r.count,
                        hash="%016x" % r.hash, atom_strategies=r.atom_strategy, atom_pairs=r.atom_pairs,
                        join_rows=r.join_rows))
    print(json.dumps({"metric": "CRPQ wall time (typed social graph)", "value": out[0]["ms"], "unit": "ms",
                      "n_gpus": 1, "higher_is_better": False, "dtype": "u32", "data": "synthetic (seeded)",
                      "config": {"workload": "social_p1m_m10m_t16k: %d vertices, %d distinct edges" % (
                          el.n_vertices, g.info()["n_edges"])},
                      "ingest_ms": round(ingest_ms, 1), "cases": out}), flush=True)
    g.close()


def serve_points(g, el, seed, rates, seconds, warmup_seconds, workers, pool_gib, max_requests, burst_requests,
                 resident_slots=0, resident_iters=0):
    """Requests of synth.serve_requests arrive as a Poisson stream at each rate ('burst': all at once,
    the server's capacity); latency is scheduled arrival -> completion.  The same requests then run
    one at a time (plain FIFO, no overlap) for the edges/s comparison and to check that every result
    is the one it has alone.  With resident_slots, single-source RPQs run on the server's resident
    engine (64-source units in one persistent batched kernel that takes arrivals between launches);
    slices and CRPQs run on the worker streams.  Returns (points, every result identical to its
    result alone)."""
    import numpy as np
    import torch

    import paper_2602_20748_amd as rpq
    import synth

    ring = [torch.empty(1 << 20, dtype=torch.int64, device="cuda") for _ in range(64)]
    points = []
    identical = True
    for tok in [x for x in rates.split(",") if x]:
        burst = tok == "burst"
        qps = float("inf") if burst else float(tok)
        n = int(min(max_requests, burst_requests) if burst else
                min(max_requests, qps * (seconds + warmup_seconds)))
        reqs = synth.serve_requests(n, el.n_vertices, el.names, seed=seed + 1000)
        arrive = np.zeros(n) if burst else synth.poisson_arrivals(qps, n, seed=seed + 3000) * 1e3
        nfa = [rpq.rpq_nfa_compile(r[1], el.names) if r[0] != "crpq" else None for r in reqs]
        print("bench: serving %d requests at %s QPS" % (n, tok), file=sys.stderr, flush=True)
        srv = rpq.Server(g, int(pool_gib * (1 << 30)), workers=workers, resident_slots=resident_slots,
                         resident_width=64, resident_max_units=1, resident_iters=resident_iters)
        last_note = time.time()

        def wait(t):
            # poll rather than block, so that a long wait still reports the server's state
            nonlocal last_note
            while True:
                d = srv.poll(t)
                if d["done"]:
                    return d
                if time.time() - last_note > 10:
                    last_note = time.time()
                    st = srv.stats()
                    print("bench: waiting for request %d: completed %d, failed %d, queued %d, running %d, "
                          "pool in use %.1f GiB" % (t, st["completed"], st["failed"], st["queued"], st["running"],
                                                    st["pool_in_use"] / 2 ** 30), file=sys.stderr, flush=True)
                time.sleep(0.001)

        t0 = srv.clock_ms() + 50.0
        tickets = []
        for i, r in enumerate(reqs):
            if i >= len(ring):   # a ring of pair buffers: the request that used this one must be done
                wait(tickets[i - len(ring)])
            due = t0 + arrive[i]
            while srv.clock_ms() < due:
                time.sleep(max(0.0, min(0.002, (due - srv.clock_ms()) / 1e3)))
            if r[0] == "crpq":
                tickets.append(srv.submit_crpq(r[1], r[2], binding=r[3], arrival_ms=due))
            else:
                fl = rpq.RPQ_SPARSE if (r[0] == "rpq_single" and not resident_slots) else 0
                tickets.append(srv.submit_rpq(nfa[i], r[2], flags=fl, pairs=ring[i % len(ring)], arrival_ms=due))
            if time.time() - last_note > 10:
                last_note = time.time()
                print("bench: submitted %d / %d" % (i + 1, n), file=sys.stderr, flush=True)
        done = []
        for t in tickets:
            done.append(wait(t))
            if time.time() - last_note > 10:
                last_note = time.time()
                print("bench: completed %d / %d" % (len(done), n), file=sys.stderr, flush=True)
        sst = srv.stats()
        srv.stop()
        del srv
        torch.cuda.empty_cache()   # the pool goes back before the FIFO replay allocates its workspaces
        warm = t0 if burst else t0 + warmup_seconds * 1e3
        # requests the server could not run (e.g. a workspace beyond the pool: RPQ_ENOMEM) are reported
        # and left out of the latencies and of the one-at-a-time replay
        ok_status = (0, rpq.RPQ_EOVERFLOW)
        failed = [(reqs[i][0], int(d["status"])) for i, d in enumerate(done) if d["status"] not in ok_status]
        served = [d for d in done if d["status"] in ok_status]
        meas = [d for d in served if d["arrival_ms"] >= warm] or served
        lat = np.array([d["end_ms"] - d["arrival_ms"] for d in meas])
        span = (max(d["end_ms"] for d in meas) - min(d["arrival_ms"] for d in meas)) / 1e3
        ep = sum(d["product_edges"] for d in meas)
        # the same requests alone, one at a time
        print("bench: FIFO replay of %d requests" % len(reqs), file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        fifo_s = 0.0
        fifo_ep = 0
        fifo_times = []
        for i, (r, d) in enumerate(zip(reqs, done)):
            if time.time() - last_note > 10:
                last_note = time.time()
                print("bench: FIFO %d / %d" % (i + 1, n), file=sys.stderr, flush=True)
            if d["status"] not in ok_status:
                fifo_times.append(float("nan"))
                continue
            t = time.perf_counter()
            if r[0] == "crpq":
                a = rpq.crpq_eval(g, r[1], r[2], binding=r[3])
                ok = (a.count, a.hash) == (d["count"], d["hash"])
                e = 0
            else:
                fl = rpq.RPQ_SPARSE if (r[0] == "rpq_single" and not resident_slots) else 0
                a = rpq.rpq_eval(g, nfa[i], r[2], flags=fl, pairs=ring[0], allow_overflow=True)
                ok = (a.count, a.hash, a.product_edges) == (d["count"], d["hash"], d["product_edges"])
                e = a.product_edges
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            fifo_times.append(dt)
            identical &= ok
            if d["arrival_ms"] >= warm or len(meas) == len(served):
                fifo_s += dt
                fifo_ep += e
        kinds = {k: sum(1 for r in reqs if r[0] == k) for k in ("rpq_single", "rpq_slice", "crpq")}
        service = {k: round(float(np.mean([d["end_ms"] - d["start_ms"] for r, d in zip(reqs, done)
                                           if r[0] == k and d["status"] in ok_status] or [0.0])), 3) for k in kinds}
        fifo_kind = {k: round(1e3 * float(np.mean([t for r, t in zip(reqs, fifo_times) if r[0] == k and t == t]
                                                  or [0.0])), 3) for k in kinds}
        points.append(dict(qps="burst" if burst else qps, requests=n, measured=len(meas), mix=kinds, workers=workers,
                           failed=len(failed), failed_kind_status=failed,
                           resident=dict(slots=resident_slots, completed=sst["resident_completed"],
                                         launches=sst["resident_launches"],
                                         gib=round(sst["resident_bytes"] / 2 ** 30, 2)),
                           service_ms_by_kind=service, fifo_ms_by_kind=fifo_kind,
                           p50_ms=round(float(np.percentile(lat, 50)), 3), p99_ms=round(float(np.percentile(lat, 99)), 3),
                           completed_per_s=round(len(meas) / span, 2), served_edges_per_s=ep / span,
                           fifo_edges_per_s=fifo_ep / fifo_s if fifo_s > 0 else None,
                           # below capacity the served rate is the offered load; the ratio means
                           # something only when every request is waiting at once
                           served_over_fifo=((ep / span) / (fifo_ep / fifo_s))
                           if burst and fifo_s > 0 and fifo_ep else None))
        print("bench: %s" % json.dumps(points[-1]), file=sys.stderr, flush=True)
        g.release_workspace()
        torch.cuda.empty_cache()
    return points, identical


def serve_main(args):
    """The serving sweep over --qps on its own JSON line."""
    import paper_2602_20748_amd as rpq
    import synth

    spec = synth.WORKLOADS[args.workload]
    el = synth.workload_graph(args.workload)
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, flags=rpq.RPQ_BUILD_IN_CSR,
                             names=el.names)
    points, identical = serve_points(g, el, spec["seed"], args.qps, args.serve_seconds, args.serve_warmup_seconds,
                                     args.serve_workers, args.serve_pool_gib, args.serve_max_requests,
                                     args.serve_max_requests, resident_slots=args.serve_resident_slots,
                                     resident_iters=args.serve_resident_iters)
    line = {
        "metric": "p99 latency (serving)", "value": points[-1]["p99_ms"] if points else None, "unit": "ms",
        "n_gpus": 1, "higher_is_better": False, "dtype": "u64", "data": "synthetic (seeded R-MAT; Poisson arrivals)",
        "config": {"workload": "%s serving: %d workers, %d resident slots, %.0f GiB pool" % (
            args.workload, args.serve_workers, args.serve_resident_slots, args.serve_pool_gib)},
        "results_identical_to_alone": identical, "points": points,
    }
    print(json.dumps(line), flush=True)
    g.close()


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
    import oracle
    import synth
    threads = host_cores()
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
        n = min(el.n_vertices, n * 2)
    # the same oracle on one thread, over the first sixteenth of the sample
    src1 = src[: max(1, n // 16)]
    t0 = time.perf_counter()
    e1 = 0
    for q in queries:
        e1 += oracle.rpq(og, q, sources=src1, pairs=False, threads=1).product_edges
    dt1 = time.perf_counter() - t0
    return dict(value=eprod / dt, unit="product-graph edges/s", cores=threads, kind="oracle",
                pairs_per_s=pairs / dt, single_thread_value=e1 / dt1, host_cpu=host_cpu_model(),
                host_logical_cpus=os.cpu_count(),
                sample="%d seeded sources (of %d) x %d queries, %.1f s, %d product edges; single thread: first %d "
                       "of them, %.1f s" % (n, el.n_vertices, len(queries), dt, eprod, src1.size, dt1))


def host_cores():
    """Logical CPUs this process may run on (its affinity set), i.e. every host core it is given."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except (AttributeError, OSError):
        return max(1, os.cpu_count() or 1)


def expand_roofline(prof):
    """Bytes per launch of the level expansion from its exact device tallies.

    method: the unit of work the method defines (one product edge examined, bit-parallel over the
      unit's sources): 4 B neighbour id per item, 16 B per work segment (the row offsets), 8 B per
      frontier word read, one 8 B read of the target's visited word per item-word, and 8 B per OR
      into the next frontier.
    impl: what this kernel moves on purpose -- the same plus 8 B per access beyond the method's: the
      next-frontier word read beside each visited word (two-read scheme); the seen-OR scheme makes
      the method's accesses only."""
    launches = max(1, prof["expand_launches"])
    method = (4 * prof["edge_items"] + 16 * prof["descriptors"] + 8 * prof["row_words"] + 8 * prof["word_reads"]
              + 8 * prof["word_updates"]) / launches
    impl = method + 8 * prof["expand_extra_words"] / launches
    avg_ms = prof["expand_ms"] / launches
    return method, impl, avg_ms


def other_rooflines(prof):
    """Method bytes and HBM fraction of the two other level-step kernels, from their exact tallies.

    finalize (timed with the compaction that feeds it, one pair per level): 8 B per row id (written by
      compaction, read by finalize); per row word 16 B (Next or, with seen OR, the previous level's
      visited copy read, frontier write); per non-zero word 8 B more to clear Next or advance the
      copy; 8 B per finalize access to the visited bitmap (two reads: a read and a write of each
      non-zero word; seen OR: a read of each row word); per non-zero word of a
      final-state row 16 B for the answer word.  The touch bitmap compaction scans (one bit per row) is left out;
      the tallies include the seeding finalize of each group (one row per source), which is not timed.
    extract (count passes, timed on the extraction stream): 8 B per answer word read."""
    out = {}
    fl = prof["finalize_launches"]
    if fl and prof["finalize_ms"] / fl > 1e-6:
        b = (8 * prof["finalize_rows"] + 16 * prof["finalize_row_words"] + 8 * prof["finalize_words"]
             + 8 * prof["finalize_vis_words"] + 16 * prof["finalize_ans_words"]) / fl
        ms = prof["finalize_ms"] / fl
        a = b / (ms / 1e3) / 1e9
        out["finalize"] = dict(bound="hbm", achieved=round(a, 2), peak=HBM_PEAK_GBPS, unit="GB/s",
                               frac=round(a / HBM_PEAK_GBPS, 5), avg_launch_ms=round(ms, 5), launches=fl,
                               alg_bytes_per_launch=round(b, 1), kernel="k_compact + k_finalize",
                               counters={k: prof[k] for k in ("finalize_rows", "finalize_row_words", "finalize_words",
                                                              "finalize_vis_words", "finalize_ans_words")})
    xl = prof["extract_launches"]
    if xl and prof["extract_ms"] / xl > 1e-6:
        b = 8 * prof["extract_words"] / xl
        ms = prof["extract_ms"] / xl
        a = b / (ms / 1e3) / 1e9
        out["extract"] = dict(bound="hbm", achieved=round(a, 2), peak=HBM_PEAK_GBPS, unit="GB/s",
                              frac=round(a / HBM_PEAK_GBPS, 5), avg_launch_ms=round(ms, 5), launches=xl,
                              alg_bytes_per_launch=round(b, 1), kernel="k_extract (count pass)")
    return out


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def load_traffic(path, kernel, source_files, tag):
    """Measured HBM bytes per launch, valid only for the kernel sources and the workload
    (tag = workload name, source count, queries) it was taken with."""
    import hashlib
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        h = hashlib.sha256()
        for f in source_files:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        ent = d.get(kernel)
        if not ent or ent.get("sources_sha256") != h.hexdigest() or ent.get("tag") != tag:
            return None
        return ent.get("bytes_per_launch")
    except Exception:
        return None


def mixes(g, el, seed, kinds=("single_source_256", "mixed_128_single_128_slices"), autotune=True):
    """Batched vs plain where batching is meant to pay: 256 single-source queries, and 128
    single-source queries with 128 all-pairs queries over 4,096-source slices (generated regexes,
    seeded).  Wall time of the plain launches one after the other vs one batched run (plan from the
    autotuner, graph captured on a first run); results must be identical."""
    import numpy as np
    import torch

    import paper_2602_20748_amd as rpq
    import synth

    out = {}
    for kind in kinds:
        mix = synth.rmat_query_mix(256, el.n_vertices, el.names, seed=seed + 1000, slice_width=4096)
        if kind.startswith("single"):
            rng = np.random.default_rng(seed + 2000)
            mix = [(rx, np.array([int(rng.integers(0, el.n_vertices))], np.uint32)) for rx, _ in mix]
        nfas = [rpq.rpq_nfa_compile(rx, el.names) for rx, _ in mix]
        print("bench: mix %s" % kind, file=sys.stderr, flush=True)
        res = []
        for rep in range(2):   # the first pass warms the workspaces
            res = []
            eprod = 0
            torch.cuda.synchronize()
            t = time.perf_counter()
            for nfa, (_, src) in zip(nfas, mix):
                r = rpq.rpq_eval(g, nfa, src)
                res.append((r.count, r.hash, r.product_edges))
                eprod += r.product_edges
            torch.cuda.synchronize()
            t_plain = time.perf_counter() - t
        b = rpq.rpq_batch_create(g)
        for nfa, (_, src) in zip(nfas, mix):
            b.add(nfa, src)
        tuned = b.autotune() if autotune else None
        b.run()
        torch.cuda.synchronize()
        t = time.perf_counter()
        b.run()
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t
        st = b.stats()
        same = all((b.result(i).count, b.result(i).hash, b.result(i).product_edges) == res[i] for i in range(len(mix)))
        out[kind] = dict(queries=len(mix), product_edges=eprod, plain_ms=round(t_plain * 1e3, 2),
                         batched_ms=round(t_batch * 1e3, 2), batched_over_plain=round(t_plain / t_batch, 3),
                         results_identical=same, plan=dict(batch_width=st["batch_width"], slots=st["slots"],
                                                            units=st["n_units"], tuned=tuned))
        b.close()
    return out


def plans_main(args):
    """The paper's Q5 shape a.b.c* three ways (Section 2.3; Section 8's plan comparison): the one-automaton
    plan, start in the middle (a, then b.c* from a's targets, materialized and joined) and loop cache
    (a.b, then c* from its targets).  Same sources, same keys; time per plan over the timed runs."""
    import numpy as np
    import torch

    import paper_2602_20748_amd as rpq
    import synth

    name = args.workload
    spec = synth.WORKLOADS[name]
    print("bench: generating %s" % name, file=sys.stderr, flush=True)
    el = synth.workload_graph(name)
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    n_src = 4096 if args.sources < 0 else args.sources
    src = synth.sample_sources(el.n_vertices, n_src, seed=spec["seed"] + 2000)
    src_dev = torch.from_numpy(src.astype(np.int64)).to(torch.int32).cuda()
    comp = lambda rx: rpq.rpq_nfa_compile(rx, el.names)
    plans = {
        "one automaton a.b.c*": lambda: (rpq.rpq_eval(g, comp("a.b.c*"), src_dev), None),
        "start in the middle a | b.c*": lambda: rpq.rpq_eval_split(g, comp("a"), comp("b.c*"), src_dev),
        "loop cache a.b | c*": lambda: rpq.rpq_eval_split(g, comp("a.b"), comp("c*"), src_dev),
    }
    runs = max(1, min(args.steps, 5))
    out = {}
    for pname, fn in plans.items():
        print("bench: plan %s" % pname, file=sys.stderr, flush=True)
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(runs):
            res, info = fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / runs
        out[pname] = dict(ms=round(ms, 3), count=res.count, hash="%016x" % res.hash, info=info)
    base = out["one automaton a.b.c*"]
    identical = all((v["count"], v["hash"]) == (base["count"], base["hash"]) for v in out.values())
    best = min(v["ms"] for k, v in out.items() if k != "one automaton a.b.c*")
    line = {"metric": "split plan vs one-automaton plan (a.b.c*)", "value": round(base["ms"] / best, 3), "unit": "x",
            "n_gpus": 1, "higher_is_better": True, "dtype": "u64", "data": "synthetic (seeded R-MAT; no dataset)",
            "config": {"workload": "%s: %d vertices, %d distinct edges, %d labels; %d seeded sampled sources; "
                                   "%d timed runs per plan" % (name, el.n_vertices, g.info()["n_edges"], el.n_labels,
                                                               n_src, runs)},
            "plans": out, "results_identical": identical}
    print(json.dumps(line), flush=True)
    g.close()


def mix_main(args):
    """The 256-query batch on R-MAT scale 22 (half single-source queries, half all-pairs over
    4,096-source slices; generated regexes, 2-12 automaton states): the batched persistent launch,
    plan from the autotuner, against the same queries as plain launches one after the other."""
    import torch

    import paper_2602_20748_amd as rpq
    import synth

    name = "rmat22_l16"
    spec = synth.WORKLOADS[name]
    print("bench: generating %s" % name, file=sys.stderr, flush=True)
    el = synth.workload_graph(name)
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    out = mixes(g, el, spec["seed"], kinds=("mixed_128_single_128_slices",), autotune=not args.no_autotune)
    m = out["mixed_128_single_128_slices"]
    line = {"metric": "batched vs plain (256-query mix)", "value": m["batched_over_plain"], "unit": "x",
            "n_gpus": 1, "higher_is_better": True, "dtype": "u64", "data": "synthetic (seeded R-MAT; no dataset)",
            "config": {"workload": "%s: R-MAT scale 22, %d vertices, %d distinct edges, 16 labels; 256 generated "
                                   "queries, 128 single-source + 128 over 4,096-source slices" % (
                                       name, el.n_vertices, g.info()["n_edges"])},
            "mix": m}
    print(json.dumps(line), flush=True)
    g.close()
    torch.cuda.synchronize()


def main():
    args = parse_args()
    if args.gpus != 1:
        print("bench.py: the benchmark runs on exactly one GPU (one MI355X); --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
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
    if args.serve:
        serve_main(args)
        return
    if args.crpq:
        crpq_main()
        return
    if args.mix:
        mix_main(args)
        return
    if args.plans:
        plans_main(args)
        return
    spec = synth.WORKLOADS[args.workload]
    queries = spec.get("queries", [])
    if args.queries:
        queries = [q for q in args.queries.split(",") if q]
    if not queries:
        print("bench.py: workload %s has no default queries; pass --queries" % args.workload, file=sys.stderr)
        sys.exit(2)
    n_sample = spec.get("bench_sources", 0) if args.sources < 0 else args.sources
    all_pairs = n_sample == 0
    # the R-MAT 18 all-pairs step also times the batched form of the same five queries and the mixes;
    # the sampled large-graph step times a single-source batch and a serving leg instead
    full_legs = not args.only and not args.queries
    print("bench: generating %s" % args.workload, file=sys.stderr, flush=True)
    el = synth.workload_graph(args.workload)
    serve_leg = full_legs and not all_pairs and not args.no_serve_leg
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels,
                             flags=rpq.RPQ_BUILD_IN_CSR if serve_leg else 0, names=el.names)
    info = g.info()
    src_host = None if all_pairs else synth.sample_sources(el.n_vertices, n_sample, spec["seed"] + 1000)
    src_dev = torch.from_numpy(src_host.view("int32").copy()).cuda() if src_host is not None else None
    n_src = el.n_vertices if src_host is None else int(src_host.size)
    traffic_tag = "%s|%s|%s" % (args.workload, "all" if src_host is None else n_src, ",".join(queries))
    traffic_file = args.traffic_file or os.path.join(ROOT, "profiles", "traffic_%s.json" % args.workload)
    stream = torch.cuda.current_stream()
    forms = {}

    # ------------------------------------------------------------------ plain form
    if args.only in ("", "plain"):
        opts = dict(batch_width=args.batch_width, concurrency=args.concurrency, sync_every=args.sync_every,
                    chunk_edges=args.chunk_edges,
                    visit={"auto": 0, "two-reads": rpq.RPQ_VISIT_TWO_READS, "seen-or": rpq.RPQ_VISIT_SEEN_OR}[args.visit])
        per_source = torch.zeros((n_src, 2), dtype=torch.int64, device="cuda")
        qtimes = {q: 0.0 for q in queries}

        def step():
            out = []
            for q in queries:
                t = time.perf_counter()
                nfa = rpq.rpq_nfa_compile(q, el.names)
                out.append(rpq.rpq_eval(g, nfa, src_dev, opts=opts, per_source=per_source))
                qtimes[q] += time.perf_counter() - t
            return out

        for i in range(args.warmup):
            print("bench: plain warmup %d" % i, file=sys.stderr, flush=True)
            step()
        torch.cuda.synchronize()
        for q in queries:
            qtimes[q] = 0.0
        rpq.rpq_profile_read(reset=True)
        rpq.rpq_profile_enable(True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        eprod = pairs = 0
        per_query = {}
        torch.cuda.synchronize()
        ev0.record(stream)
        for i in range(args.steps):
            for q, r in zip(queries, step()):
                eprod += r.product_edges
                pairs += r.count
                per_query[q] = dict(count=r.count, hash="%016x" % r.hash, product_edges=r.product_edges,
                                    levels=r.levels, max_depth=r.max_depth)
            print("bench: plain step %d done" % i, file=sys.stderr, flush=True)
        ev1.record(stream)
        torch.cuda.synchronize()
        rpq.rpq_profile_enable(False)
        prof = rpq.rpq_profile_read(reset=True)
        secs = ev0.elapsed_time(ev1) / 1e3
        for q in queries:
            per_query[q]["ms"] = round(qtimes[q] * 1e3 / max(1, args.steps), 3)
        # dominant kernel of the plain form: the level expansion, timed by HIP events on the stream
        # it is launched on; bytes from its exact tallies (expand_roofline)
        method, impl, avg_ms = expand_roofline(prof)
        achieved = method / (avg_ms / 1e3) / 1e9 if avg_ms > 0 else 0.0
        achieved_impl = impl / (avg_ms / 1e3) / 1e9 if avg_ms > 0 else 0.0
        step_rooflines = other_rooflines(prof)
        forms["plain"] = dict(
            step_rooflines=step_rooflines,
            value=eprod / secs, ms_per_step=secs * 1e3 / args.steps, distinct_pairs_per_s=pairs / secs,
            per_query=per_query,
            roofline=dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBPS, unit="GB/s",
                          frac=round(achieved / HBM_PEAK_GBPS, 5),
                          traffic=load_traffic(traffic_file, "k_expand",
                                               ["paper_2602_20748_amd/csrc/eval.hip"], traffic_tag),
                          kernel="k_expand", traffic_tag=traffic_tag,
                          bytes_rule="method: 4 B/item + 16 B/segment + 8 B/frontier word + 8 B/visited-word "
                                     "read + 8 B/OR",
                          avg_launch_ms=round(avg_ms, 5), launches=prof["expand_launches"],
                          alg_bytes_per_launch=round(method, 1),
                          impl_bytes_per_launch=round(impl, 1), achieved_impl=round(achieved_impl, 2),
                          frac_impl=round(achieved_impl / HBM_PEAK_GBPS, 5),
                          finalize_avg_ms=round(prof["finalize_ms"] / max(1, prof["finalize_launches"]), 5),
                          counters={k: prof[k] for k in ("expand_launches", "edge_items", "descriptors", "row_words",
                                                         "word_reads", "word_updates", "expand_extra_words",
                                                         "expand_ms", "finalize_ms")},
                          visit=(args.visit if args.visit != "auto"
                                 else "seen-or" if el.n_vertices >= (1 << 22) else "two-reads")))

    # ------------------------------------------------------------------ batched form
    g.release_workspace()
    torch.cuda.empty_cache()
    if args.only == "batched" or (full_legs and all_pairs):
        plan_opts = None
        if args.batched_plan:
            w_, h_ = (int(x) for x in args.batched_plan.split(":"))
            plan_opts = dict(batch_width=w_, chunk_edges=h_)
        b = rpq.rpq_batch_create(g, opts=plan_opts)
        for q in queries:
            b.add(rpq.rpq_nfa_compile(q, el.names), src_dev, per_source=True)
        tuned = None
        if not args.no_autotune and plan_opts is None:
            print("bench: autotuning the batch", file=sys.stderr, flush=True)
            tuned = b.autotune()
        plan_chunk = (tuned or {}).get("chunk_edges") or (plan_opts or {}).get("chunk_edges") or 16
        for i in range(args.warmup):
            print("bench: batched warmup %d" % i, file=sys.stderr, flush=True)
            b.run()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        eprod = pairs = 0
        kernel_ms = 0.0
        tally = dict(edge_items=0, descriptors=0, word_reads=0, word_updates=0, finalized_rows=0,
                     finalized_words=0, iterations=0)
        per_query = {}
        ev0.record(stream)
        for i in range(args.steps):
            b.run()
            st = b.stats()
            kernel_ms += st["last_kernel_ms"]
            for k in tally:
                tally[k] += st[k]
            for qi, q in enumerate(queries):
                r = b.result(qi)
                eprod += r.product_edges
                pairs += r.count
                per_query[q] = dict(count=r.count, hash="%016x" % r.hash, product_edges=r.product_edges)
            print("bench: batched step %d done" % i, file=sys.stderr, flush=True)
        ev1.record(stream)
        torch.cuda.synchronize()
        secs = ev0.elapsed_time(ev1) / 1e3
        st = b.stats()
        K = st["row_words"]
        # dominant kernel of the batched form: the persistent kernel (one launch per step).
        # Method bytes = expansion (as in the plain form: one 8 B visited-word read per item-word)
        # + finalize (per row: 4 B id, 8K B next read, 8K B frontier-row write, 12 B label mask and
        # slot; per non-zero word: 8 B next clear + 16 B visited OR; 16 B per descriptor written)
        # + compaction (8 B per touch word scanned per iteration, 4 B per row id).
        exp = (4 * tally["edge_items"] + 16 * tally["descriptors"] + 8 * K * tally["descriptors"]
               + 8 * tally["word_reads"] + 8 * tally["word_updates"])
        fin = tally["finalized_rows"] * (4 + 16 * K + 12) + 24 * tally["finalized_words"] + 16 * tally["descriptors"]
        cmp_ = 8 * tally["iterations"] * st["touch_words"] + 4 * tally["finalized_rows"]
        alg = (exp + fin + cmp_) / max(1, args.steps)
        kms = kernel_ms / max(1, args.steps)
        achieved = alg / (kms / 1e3) / 1e9 if kms > 0 else 0.0
        forms["batched"] = dict(
            value=eprod / secs, ms_per_step=secs * 1e3 / args.steps, distinct_pairs_per_s=pairs / secs,
            per_query=per_query, plan=dict(batch_width=st["batch_width"], slots=st["slots"], units=st["n_units"],
                                           blocks=st["blocks"], tuned=tuned,
                                           iterations_per_step=tally["iterations"] // max(1, args.steps),
                                           phase_ms_last_step=st["phase_ms"]),
            roofline=dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBPS, unit="GB/s",
                          frac=round(achieved / HBM_PEAK_GBPS, 5),
                          traffic=load_traffic(traffic_file, "k_batch",
                                               ["paper_2602_20748_amd/csrc/batch.hip",
                                                "paper_2602_20748_amd/csrc/internal.h"],
                                               "%s|plan=%d:%d" % (traffic_tag, st["batch_width"], plan_chunk)),
                          traffic_tag="%s|plan=%d:%d" % (traffic_tag, st["batch_width"], plan_chunk),
                          kernel="k_batch", avg_launch_ms=round(kms, 3), launches=args.steps,
                          alg_bytes_per_launch=round(alg, 1),
                          counters={k: v // max(1, args.steps) for k, v in tally.items()}))
        b.close()

    mix_results = None
    if full_legs:
        g.release_workspace()
        torch.cuda.empty_cache()
        kinds = ("single_source_256", "mixed_128_single_128_slices") if all_pairs else ("single_source_256",)
        if not args.no_mixes:
            mix_results = mixes(g, el, spec["seed"], kinds=kinds)
    serving = None
    if serve_leg:
        g.release_workspace()
        torch.cuda.empty_cache()
        points, identical = serve_points(g, el, spec["seed"], args.serve_leg, args.serve_leg_seconds, 2.0,
                                         args.serve_workers, args.serve_pool_gib, args.serve_max_requests,
                                         args.serve_leg_burst, resident_slots=args.serve_resident_slots,
                                         resident_iters=args.serve_resident_iters)
        serving = dict(points=points, results_identical_to_alone=identical,
                       p50_ms={str(p["qps"]): p["p50_ms"] for p in points},
                       p99_ms={str(p["qps"]): p["p99_ms"] for p in points},
                       served_edges_per_s={str(p["qps"]): p["served_edges_per_s"] for p in points},
                       fifo_edges_per_s={str(p["qps"]): p["fifo_edges_per_s"] for p in points})
    form = args.form if args.form in forms else next(iter(forms))
    main_form = forms[form]
    cpu = None
    if args.cpu_baseline_seconds > 0:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(el, queries, args.cpu_baseline_seconds)
    batched_over_plain = None
    if "batched" in forms and "plain" in forms:
        batched_over_plain = forms["batched"]["value"] / forms["plain"]["value"]
    elif mix_results:
        batched_over_plain = mix_results["single_source_256"]["batched_over_plain"]
    line = {
        "metric": "product-graph edges/sec",
        "value": main_form["value"],
        "unit": "product-graph edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_form["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (seeded R-MAT; no dataset)",
        "config": {"workload": "%s: %s, %d vertices, %d drawn / %d distinct edges, %d labels Zipf(%g);"
                               " %s %s; %s form"
                               % (args.workload, describe_graph(spec), el.n_vertices, el.n_edges, info["n_edges"],
                                  el.n_labels, spec.get("zipf_s", 1.1),
                                  "all-pairs" if src_host is None else
                                  "%d seeded sampled sources (seed %d)," % (n_src, spec["seed"] + 1000),
                                  ", ".join(queries), form),
                   "sources": n_src, "queries": queries, "form": form},
        "distinct_pairs_per_s": main_form["distinct_pairs_per_s"],
        "batched_over_plain": batched_over_plain,
        "batched_vs_plain_mixes": mix_results,
        "serving": serving,
        "forms": {k: {kk: vv for kk, vv in v.items() if kk not in ("roofline", "step_rooflines")}
                  for k, v in forms.items()},
        "roofline": main_form["roofline"],
        "roofline_other": dict({k: v["roofline"] for k, v in forms.items() if k != form},
                               **(forms["plain"].get("step_rooflines") or {}) if "plain" in forms else {}),
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    g.close()


if __name__ == "__main__":
    main()
