"""GPU parity of length-bounded RPQs (only walks of at most k edges count; the extension named in
the paper's conclusion) against the oracle's bounded search, in every form: the bit-parallel plain
form at several unit widths, the per-source hash-set search (RPQ_SPARSE), reverse walks and the
batched persistent kernel.  Keys, counts, checksums, per-source tallies and product edges (edges of
expanded product vertices only) are compared bit-exactly."""
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


def keys_np(t):
    return t.cpu().numpy().view(np.uint64)


def check(rpq, g, og, regex, sources, k, flags=0, opts=None, names=None):
    names = names or og.names
    nfa = rpq.rpq_nfa_compile(regex, names)
    res = rpq.rpq_eval(g, nfa, sources, flags=flags, opts=opts, pairs=True, per_source=True, max_length=k)
    want = oracle.rpq(og, regex, sources=sources, max_length=k)
    assert res.count == want.count, (regex, k, res.count, want.count)
    assert np.array_equal(keys_np(res.pairs), want.pairs), (regex, k)
    assert res.hash == want.hash, (regex, k)
    assert res.product_edges == want.product_edges, (regex, k, res.product_edges, want.product_edges)
    assert np.array_equal(keys_np(res.per_source), want.per_source), (regex, k)
    return res, want


def test_bounded_random_graphs_every_form(rpq):
    rng = np.random.default_rng(3101)
    names = ["a", "b", "c", "d"]
    for trial in range(12):
        n = int(rng.integers(20, 400))
        m = int(rng.integers(n, 6 * n))
        src = rng.integers(0, n, size=m).astype(np.uint32)
        dst = rng.integers(0, n, size=m).astype(np.uint32)
        lab = rng.integers(0, 4, size=m).astype(np.uint8)
        g = rpq.rpq_graph_create(src, lab, dst, n, 4, flags=rpq.RPQ_BUILD_IN_CSR, names=names)
        og = oracle.OracleGraph(n, src, lab, dst, 4, names)
        sources = np.sort(rng.choice(n, size=int(rng.integers(1, n + 1)), replace=False)).astype(np.uint32)
        for q in range(3):
            rx = synth.random_regex(rng, names, max_leaves=6)
            for k in (0, 1, 2, 3, 5, 40):
                say("case: bounded trial=%d n=%d m=%d %s k=%d" % (trial, n, m, rx, k))
                check(rpq, g, og, rx, sources, k)
                check(rpq, g, og, rx, sources, k, opts=dict(batch_width=64, concurrency=1))
                check(rpq, g, og, rx, sources, k, opts=dict(batch_width=128, visit=rpq.RPQ_VISIT_SEEN_OR))
                check(rpq, g, og, rx, sources, k, flags=rpq.RPQ_SPARSE)
        g.close()


def test_bounded_large_bound_equals_unbounded_and_is_monotone(rpq):
    el = synth.workload_graph("uniform_v1000_e5000_l4")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    nfa = rpq.rpq_nfa_compile("a.b.c*", el.names)
    full = rpq.rpq_eval(g, nfa, None, pairs=True)
    prev = -1
    for k in range(0, full.max_depth + 3):
        say("case: uniform a.b.c* k=%d" % k)
        r = rpq.rpq_eval(g, nfa, None, pairs=True, max_length=k)
        assert r.count >= prev
        prev = r.count
        if k >= full.max_depth:
            assert (r.count, r.hash, r.product_edges) == (full.count, full.hash, full.product_edges)
            assert np.array_equal(keys_np(r.pairs), keys_np(full.pairs))
    g.close()


def test_bounded_reverse_matches_transposed_graph(rpq):
    rng = np.random.default_rng(3102)
    names = ["a", "b", "c"]
    n, m = 300, 1200
    src = rng.integers(0, n, size=m).astype(np.uint32)
    dst = rng.integers(0, n, size=m).astype(np.uint32)
    lab = rng.integers(0, 3, size=m).astype(np.uint8)
    g = rpq.rpq_graph_create(src, lab, dst, n, 3, flags=rpq.RPQ_BUILD_IN_CSR, names=names)
    # walks of the reversed language on the transposed graph are the walks of the query backwards
    ogt = oracle.OracleGraph(n, dst, lab, src, 3, names)
    sources = np.arange(0, n, 3, dtype=np.uint32)
    for rx, rrx in (("a.b*", "b*.a"), ("(a|b).c.a", "a.c.(a|b)"), ("a*.b", "b.a*")):
        for k in (1, 2, 4):
            say("case: bounded reverse %s k=%d" % (rx, k))
            nfa = rpq.rpq_nfa_compile(rx, names)
            got = rpq.rpq_eval(g, nfa, sources, flags=rpq.RPQ_REVERSE, pairs=True, max_length=k)
            want = oracle.rpq(ogt, rrx, sources=sources, max_length=k)
            assert np.array_equal(keys_np(got.pairs), want.pairs), (rx, k)
            assert (got.count, got.hash) == (want.count, want.hash), (rx, k)
    g.close()


def test_bounded_batched_matches_plain_and_oracle(rpq):
    rng = np.random.default_rng(3103)
    names = ["a", "b", "c", "d"]
    n, m = 2000, 9000
    src = rng.integers(0, n, size=m).astype(np.uint32)
    dst = rng.integers(0, n, size=m).astype(np.uint32)
    lab = rng.integers(0, 4, size=m).astype(np.uint8)
    g = rpq.rpq_graph_create(src, lab, dst, n, 4, names=names)
    og = oracle.OracleGraph(n, src, lab, dst, 4, names)
    qs = []
    for i in range(24):
        rx = synth.random_regex(rng, names, max_leaves=6)
        lo = int(rng.integers(0, n - 300))
        s = np.arange(lo, lo + int(rng.integers(1, 300)), dtype=np.uint32)
        k = [0, 1, 2, 3, 6, None][i % 6]
        qs.append((rx, s, k))
    for width, visit in ((64, 0), (256, 0), (128, rpq.RPQ_VISIT_SEEN_OR)):
        say("case: bounded batch width %d visit %d" % (width, visit))
        b = rpq.rpq_batch_create(g, opts=dict(batch_width=width, slots=3, visit=visit))
        for rx, s, k in qs:
            b.add(rpq.rpq_nfa_compile(rx, names), s, pairs_capacity=1 << 20, per_source=True, max_length=k)
        b.run()
        for i, (rx, s, k) in enumerate(qs):
            r = b.result(i)
            want = oracle.rpq(og, rx, sources=s, max_length=k)
            assert (r.count, r.hash, r.product_edges) == (want.count, want.hash, want.product_edges), (rx, k)
            assert np.array_equal(keys_np(r.pairs), want.pairs), (rx, k)
            assert np.array_equal(keys_np(r.per_source), want.per_source), (rx, k)
        b.close()
    g.close()


@pytest.mark.parametrize("regex", ["a*", "a.b*", "(a.b)*"])
def test_bounded_rmat18_sampled_sources(rpq, regex):
    el = synth.workload_graph("rmat18_l8")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    og = oracle.OracleGraph.from_edgelist(el)
    src = synth.sample_sources(el.n_vertices, 256, seed=3104)
    for k in (1, 3, 6):
        say("case: bounded rmat18 %s k=%d" % (regex, k))
        check(rpq, g, og, regex, src, k)
        check(rpq, g, og, regex, src, k, opts=dict(visit=rpq.RPQ_VISIT_SEEN_OR))
    g.close()


def test_bounded_invalid_arguments(rpq):
    el = synth.workload_graph("uniform_v1000_e5000_l4")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    nfa = rpq.rpq_nfa_compile("a*", el.names)
    with pytest.raises(rpq.RpqError) as e:   # the flag without its options
        rpq.rpq_eval(g, nfa, np.array([1, 2], np.uint32), flags=rpq.RPQ_LENGTH_BOUND)
    assert e.value.code == rpq.RPQ_EINVAL
    b = rpq.rpq_batch_create(g)
    b.add(nfa, np.array([1, 2], np.uint32))
    with pytest.raises(rpq.RpqError) as e:   # unknown query
        rpq.rpq_batch_bound_length(b, 5, 3)
    assert e.value.code == rpq.RPQ_EINVAL
    b.close()
    g.close()
