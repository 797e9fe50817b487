"""GPU tests of the serving loop (rpq_serve_*): every request's result in a mixed stream equals
the CPU oracle's (Definitions 1 and 2) and its result alone, requests overlap on the device, and
memory pressure only changes the schedule."""
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rpq():
    import torch
    import paper_2602_20748_amd as m
    assert torch.cuda.is_available()
    m.load_library()
    return m


@pytest.fixture(scope="module")
def rmat18(rpq):
    el = synth.workload_graph("rmat18_l8")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, flags=rpq.RPQ_BUILD_IN_CSR,
                             names=el.names)
    yield el, g
    g.close()


@pytest.fixture(scope="module")
def og18(rmat18):
    return oracle.OracleGraph.from_edgelist(rmat18[0])


def oracle_threads():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except (AttributeError, OSError):
        return 8


def oracle_result(og, item):
    """The oracle's (count, checksum, product edges or None, sorted keys or None) of one request:
    full keys for single-source RPQs, count and checksum for slices, the tuple set of a CRPQ."""
    T = oracle_threads()
    if item[0] == "crpq":
        _, atoms, nv, binding = item
        tuples = oracle.crpq_forward(og, atoms, nv, binding=binding, threads=T)
        return (len(tuples), oracle.crpq_hash(tuples), None, None)
    kind, rx, src = item
    if src.size == 1:
        w = oracle.rpq(og, rx, sources=src, threads=T)
        return (w.count, w.hash, w.product_edges, w.pairs)
    w = oracle.rpq(og, rx, sources=src, pairs=False, threads=T)
    return (w.count, w.hash, w.product_edges, None)


def request_mix(rng, el, n):
    """Single-source RPQs (sparse search), 512-source slice RPQs (bit-parallel) and 2-3 atom CRPQs
    anchored at a random source (chain, fork, triangle)."""
    mix = []
    for i in range(n):
        kind = i % 5
        rx = synth.random_regex(rng, el.names[:6], max_leaves=6)
        if kind in (0, 1):
            mix.append(("rpq_sparse", rx, np.array([int(rng.integers(0, el.n_vertices))], np.uint32)))
        elif kind in (2, 3):
            lo = int(rng.integers(0, el.n_vertices - 512))
            mix.append(("rpq_dense", rx, np.arange(lo, lo + 512, dtype=np.uint32)))
        else:
            s = int(rng.integers(0, el.n_vertices))
            r1, r2, r3 = (synth.random_regex(rng, el.names[4:8], max_leaves=3) for _ in range(3))
            shape = i % 3
            if shape == 0:      # chain s -r1-> y -r2-> z
                mix.append(("crpq", [(0, r1, 1), (1, r2, 2)], 3, [s, None, None]))
            elif shape == 1:    # fork s -r1-> y and s -r2-> y
                mix.append(("crpq", [(0, r1, 1), (0, r2, 1)], 2, [s, None]))
            else:               # triangle s -r1-> y, y -r2-> z, s -r3-> z
                mix.append(("crpq", [(0, r1, 1), (1, r2, 2), (0, r3, 2)], 3, [s, None, None]))
    return mix


def run_alone(rpq, g, el, item):
    import torch
    if item[0] == "crpq":
        _, atoms, nv, binding = item
        r = rpq.crpq_eval(g, atoms, nv, binding=binding)
        return (r.count, r.hash, None)
    kind, rx, src = item
    nfa = rpq.rpq_nfa_compile(rx, el.names)
    flags = rpq.RPQ_SPARSE if kind == "rpq_sparse" else 0
    r = rpq.rpq_eval(g, nfa, src, flags=flags, pairs=True)
    return (r.count, r.hash, r.product_edges, r.pairs.cpu().numpy().view(np.uint64).copy())


def submit(rpq, srv, el, item):
    import torch
    if item[0] == "crpq":
        _, atoms, nv, binding = item
        return srv.submit_crpq(atoms, nv, binding=binding), None
    kind, rx, src = item
    nfa = rpq.rpq_nfa_compile(rx, el.names)
    flags = rpq.RPQ_SPARSE if kind == "rpq_sparse" else 0
    buf = torch.empty(1 << 20, dtype=torch.int64, device="cuda")
    return srv.submit_rpq(nfa, src, flags=flags, pairs=buf), buf


def check_mix(rpq, g, el, mix, alone, pool_bytes, workers, want=None):
    """Serve the mix; every result must equal its result alone and, when given, the oracle's."""
    srv = rpq.Server(g, pool_bytes, workers=workers)
    sub = [submit(rpq, srv, el, it) for it in mix]
    done = [srv.wait(t) for t, _ in sub]
    st = srv.stats()
    srv.stop()
    for i, (it, (t, buf), d, a) in enumerate(zip(mix, sub, done, alone)):
        # a pair buffer smaller than the result is filled and the request reports the overflow
        assert d["status"] == 0 or (d["status"] == rpq.RPQ_EOVERFLOW and it[0] != "crpq"
                                    and d["count"] > buf.numel()), (it, d)
        if it[0] == "crpq":
            assert (d["count"], d["hash"]) == a[:2], it
        else:
            assert (d["count"], d["hash"], d["product_edges"]) == a[:3], it
            n = min(d["count"], buf.numel())
            assert np.array_equal(buf[:n].cpu().numpy().view(np.uint64), a[3][:n]), it
        if want is not None:
            w = want[i]
            assert (d["count"], d["hash"]) == (w[0], w[1]), ("oracle", it)
            if w[2] is not None:
                assert d["product_edges"] == w[2], ("oracle", it)
            if w[3] is not None:
                n = min(d["count"], buf.numel())
                assert np.array_equal(buf[:n].cpu().numpy().view(np.uint64), w[3][:n]), ("oracle", it)
    assert st["completed"] == len(mix) and st["failed"] == 0 and st["pool_in_use"] == 0
    return done, st


def max_overlap(done):
    ev = sorted([(d["start_ms"], 1) for d in done] + [(d["end_ms"], -1) for d in done])
    cur = best = 0
    for _, x in ev:
        cur += x
        best = max(best, cur)
    return best


def test_results_in_the_mix_equal_alone_and_oracle(rpq, rmat18, og18):
    el, g = rmat18
    rng = np.random.default_rng(505)
    mix = request_mix(rng, el, 40)
    alone = []
    for i, it in enumerate(mix):
        say("case: serve alone %d %s" % (i, it[:2]))
        alone.append(run_alone(rpq, g, el, it))
    want = []
    for i, it in enumerate(mix):
        say("case: serve oracle %d %s" % (i, it[:2]))
        want.append(oracle_result(og18, it))
    say("case: serve mix, 4 workers, 24 GiB pool")
    done, st = check_mix(rpq, g, el, mix, alone, 24 << 30, 4, want)
    assert max_overlap(done) >= 2          # admitted requests ran at the same time
    assert all(d["end_ms"] >= d["start_ms"] >= d["arrival_ms"] for d in done)


def test_memory_pressure_changes_only_the_schedule(rpq, rmat18, og18):
    el, g = rmat18
    rng = np.random.default_rng(506)
    mix = request_mix(rng, el, 25)   # CRPQs included: they grow their workspace through the queue
    alone = [run_alone(rpq, g, el, it) for it in mix]
    want = [oracle_result(og18, it) for it in mix]
    # the smallest pool that admits the largest single request: requests run one or two at a time,
    # and dense ones are split into fewer units in flight
    need = max(rpq.rpq_eval_workspace_size(g, rpq.rpq_nfa_compile(it[1], el.names), 512, 0,
                                           dict(batch_width=64, concurrency=1))
               for it in mix if it[0] == "rpq_dense")
    say("case: serve under pressure, pool %d bytes" % need)
    done, st = check_mix(rpq, g, el, mix, alone, int(need * 1.5), 4, want)
    assert st["pool_peak"] <= int(need * 1.5)


def test_submit_rejects(rpq, rmat18):
    el, g = rmat18
    srv = rpq.Server(g, 1 << 20, workers=2)
    nfa = rpq.rpq_nfa_compile("a*", el.names)
    with pytest.raises(rpq.RpqError) as e:   # a dense all-pairs query can never fit 1 MiB
        srv.submit_rpq(nfa, None)
    assert e.value.code == rpq.RPQ_ENOMEM
    bad = rpq.Nfa()
    with pytest.raises(rpq.RpqError) as e:
        srv.submit_rpq(bad, np.array([1], np.uint32))
    assert e.value.code == rpq.RPQ_EINVAL
    srv.stop()
    srv = rpq.Server(g, 64 << 20, workers=2)
    t = srv.submit_rpq(nfa, np.array([5, 3], np.uint32), flags=rpq.RPQ_SPARSE)   # unsorted: fails when run
    d = srv.wait(t)
    assert d["done"] and d["status"] == rpq.RPQ_EINVAL
    ok = srv.wait(srv.submit_rpq(nfa, np.array([3, 5], np.uint32), flags=rpq.RPQ_SPARSE))
    assert ok["status"] == 0 and ok["count"] > 0   # the server keeps serving after a failed request
    assert srv.stats()["failed"] == 1
    srv.stop()


def engine_takes(rpq, rx, names, states=12, succ=4):
    """The server's routing rule for the resident engine's automaton limits."""
    nfa = rpq.rpq_nfa_compile(rx, names)
    most = max(bin(int(nfa.delta[i])).count("1") for i in range(len(nfa.delta)))
    return nfa.n_states <= states and most <= succ


def test_resident_engine_admits_while_running_and_matches_oracle(rpq, rmat18, og18):
    """Dense RPQs go to the resident engine (a persistent batched kernel fed between bounded
    launches); a second wave is submitted while the first runs and joins the same device unit
    queue.  Every result equals the oracle's and the request's result alone; CRPQs and sparse
    requests run on the worker streams at the same time."""
    import time

    import torch
    el, g = rmat18
    rng = np.random.default_rng(611)
    T = oracle_threads()
    items = []
    for i in range(36):
        rx = synth.random_regex(rng, el.names[:6], max_leaves=6)
        if i % 6 == 5:
            # light CRPQs (no closures): they only have to run on the workers beside the engine
            s = int(rng.integers(0, el.n_vertices))
            if i % 12 == 5:
                items.append(("crpq", [(0, "e", 1), (1, "f|g", 2)], 3, [s, None, None]))
            else:
                items.append(("crpq", [(0, "a.b", 1), (0, "c|d", 1)], 2, [s, None]))
        elif i % 6 == 4:
            items.append(("rpq_sparse", rx, np.array([int(rng.integers(0, el.n_vertices))], np.uint32)))
        elif i % 2 == 0:
            items.append(("single", rx, np.array([int(rng.integers(0, el.n_vertices))], np.uint32)))
        else:
            lo = int(rng.integers(0, el.n_vertices - 300))
            items.append(("slice", rx, np.arange(lo, lo + 300, dtype=np.uint32)))
    want, alone = [], []
    for i, it in enumerate(items):
        say("case: resident oracle/alone %d %s" % (i, it[:2]))
        if it[0] == "crpq":
            want.append(oracle_result(og18, it))
            alone.append(run_alone(rpq, g, el, it))
            continue
        kind, rx, src = it
        w = oracle.rpq(og18, rx, sources=src, threads=T)
        want.append(w)
        nfa = rpq.rpq_nfa_compile(rx, el.names)
        a = rpq.rpq_eval(g, nfa, src, flags=rpq.RPQ_SPARSE if kind == "rpq_sparse" else 0,
                         pairs=True if kind != "slice" else None, per_source=True if kind == "slice" else None)
        alone.append(a)
    say("case: resident engine, 16 slots of 64 sources, 2 workers")
    srv = rpq.Server(g, 16 << 30, workers=2, resident_slots=16, resident_width=64, resident_iters=4)
    subs = []

    def submit_item(it):
        if it[0] == "crpq":
            _, atoms, nv, binding = it
            return srv.submit_crpq(atoms, nv, binding=binding), None, None
        kind, rx, src = it
        nfa = rpq.rpq_nfa_compile(rx, el.names)
        if kind == "slice":
            ps = torch.full((src.size, 2), -1, dtype=torch.int64, device="cuda")
            return srv.submit_rpq(nfa, src, per_source=ps), None, ps
        buf = torch.empty(1 << 20, dtype=torch.int64, device="cuda")
        flags = rpq.RPQ_SPARSE if kind == "rpq_sparse" else 0
        return srv.submit_rpq(nfa, src, flags=flags, pairs=buf), buf, None

    half = len(items) // 2
    for it in items[:half]:
        subs.append(submit_item(it))
    # the second wave arrives while the first is on the device
    t0 = time.perf_counter()
    while srv.stats()["resident_launches"] < 1 and time.perf_counter() - t0 < 30:
        time.sleep(0.0005)
    for it in items[half:]:
        subs.append(submit_item(it))
    done = [srv.wait(t) for t, _, _ in subs]
    st = srv.stats()
    srv.stop()
    say("resident stats", st)
    assert st["failed"] == 0 and st["completed"] == len(items) and st["pool_in_use"] == st["resident_bytes"]
    n_res = 0
    for it, (t, buf, ps), d, w, a in zip(items, subs, done, want, alone):
        assert d["status"] == 0, (it[:2], d)
        if it[0] == "crpq":
            assert not d["resident"]
            assert (d["count"], d["hash"]) == w[:2] == a[:2], it
            continue
        kind = it[0]
        assert d["resident"] == (kind in ("single", "slice") and engine_takes(rpq, it[1], el.names)), (kind, d)
        n_res += d["resident"]
        assert (d["count"], d["hash"], d["product_edges"]) == (w.count, w.hash, w.product_edges), it[:2]
        assert (d["count"], d["hash"], d["product_edges"]) == (a.count, a.hash, a.product_edges), it[:2]
        if kind == "slice":
            assert np.array_equal(ps.cpu().numpy().view(np.uint64), w.per_source), it[:2]
        else:
            got = buf[: d["written"]].cpu().numpy().view(np.uint64)
            assert d["written"] == d["count"]
            assert np.array_equal(got, w.pairs), it[:2]
    assert n_res == st["resident_completed"] == sum(1 for it in items if it[0] in ("single", "slice")
                                                    and engine_takes(rpq, it[1], el.names))
    assert n_res >= 20
    assert st["resident_launches"] >= 2
    # continuous admission: some second-wave request joined while a first-wave one was still running
    first_end = max(d["end_ms"] for d, it in zip(done[:half], items[:half]) if it[0] in ("single", "slice"))
    assert any(d["resident"] and d["start_ms"] < first_end for d in done[half:])


def test_resident_engine_worker_fallback_and_small_pairs(rpq):
    """On the uniform graph: automata larger than the engine's go to the workers; many single-source
    requests with pairs on the engine equal the oracle's keys."""
    import torch
    el = synth.workload_graph("uniform_v1000_e5000_l4")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    og = oracle.OracleGraph.from_edgelist(el)
    srv = rpq.Server(g, 1 << 30, workers=2, resident_slots=8, resident_width=64, resident_states=4)
    rng = np.random.default_rng(12)
    reqs = []
    for i in range(60):
        rx = ["a.b.c*", "(a|b)*.d", "a*", "a.b.c.d.a.b"][i % 4]    # the last has 7 states: workers
        src = np.array([int(rng.integers(0, el.n_vertices))], np.uint32)
        buf = torch.empty(4096, dtype=torch.int64, device="cuda")
        reqs.append((rx, src, buf, srv.submit_rpq(rpq.rpq_nfa_compile(rx, el.names), src, pairs=buf)))
    say("case: resident engine on the uniform graph, 60 single-source requests")
    for rx, src, buf, t in reqs:
        d = srv.wait(t)
        w = oracle.rpq(og, rx, sources=src)
        assert d["status"] == 0 and d["resident"] == (rx != "a.b.c.d.a.b"), (rx, d)
        assert (d["count"], d["hash"], d["product_edges"]) == (w.count, w.hash, w.product_edges), rx
        assert np.array_equal(buf[: d["written"]].cpu().numpy().view(np.uint64), w.pairs), rx
    st = srv.stats()
    srv.stop()
    assert st["failed"] == 0 and st["resident_completed"] == 45
    g.close()


def test_resident_engine_leaves_workers_a_pool_they_can_use(rpq, rmat18):
    """Worker requests are planned against the part of the pool the engine does not hold: with a pool
    only a little larger than the engine, dense requests for the workers are split to fit and finish
    (regression: they were planned against the whole pool and waited forever)."""
    import torch
    el, g = rmat18
    probe = rpq.Server(g, 4 << 30, workers=1, resident_slots=4)
    res_bytes = probe.stats()["resident_bytes"]
    probe.stop()
    rx = "a.b*"
    nfa = rpq.rpq_nfa_compile(rx, el.names)
    src = np.arange(1000, 1512, dtype=np.uint32)   # 8 units of 64: pairs go to the workers
    small = rpq.rpq_eval_workspace_size(g, nfa, src.size, rpq.RPQ_PAIRS, dict(batch_width=64, concurrency=1))
    full = rpq.rpq_eval_workspace_size(g, nfa, src.size, rpq.RPQ_PAIRS)
    pool = res_bytes + int(small * 1.5) + (1 << 20)
    assert full > pool - res_bytes     # the default plan does not fit what the workers get
    ref = rpq.rpq_eval(g, nfa, src, pairs=True)
    say("case: resident engine + a worker pool of %d bytes (default plan %d)" % (pool - res_bytes, full))
    srv = rpq.Server(g, pool, workers=1, resident_slots=4)
    buf = torch.empty(ref.count + 16, dtype=torch.int64, device="cuda")
    t = srv.submit_rpq(nfa, src, pairs=buf)
    d = srv.wait(t)
    srv.stop()
    assert d["status"] == 0 and not d["resident"]
    assert (d["count"], d["hash"], d["product_edges"]) == (ref.count, ref.hash, ref.product_edges)
    assert np.array_equal(buf[: d["written"]].cpu().numpy(), ref.pairs.cpu().numpy())
