"""GPU tests of the batched persistent form: every query of a batch must give
exactly what the plain form gives for it alone, and what the oracle gives."""
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


def keys(t):
    return t.cpu().numpy().view(np.uint64)


def plain(rpq, g, nfa, sources, want_pairs, per_source):
    return rpq.rpq_eval(g, nfa, sources, pairs=True if want_pairs else None, per_source=True if per_source else None)


def build_mix(rng, names, n_vertices, n_queries):
    mix = []
    for i in range(n_queries):
        rx = synth.random_regex(rng, names)
        kind = i % 3
        if kind == 0:
            src = np.array([int(rng.integers(0, n_vertices))], dtype=np.uint32)
            mix.append((rx, src, True, False))
        elif kind == 1:
            lo = int(rng.integers(0, max(1, n_vertices - 300)))
            src = np.arange(lo, min(n_vertices, lo + int(rng.integers(1, 300))), dtype=np.uint32)
            mix.append((rx, src, False, True))
        else:
            src = synth.sample_sources(n_vertices, int(rng.integers(1, 200)), seed=int(rng.integers(0, 1 << 30)))
            mix.append((rx, src, True, True))
    return mix


def check_batch(rpq, g, el, mix, opts, og=None, runs=2):
    b = rpq.rpq_batch_create(g, opts)
    qids = []
    expect = []
    for (rx, src, want_pairs, per_source) in mix:
        nfa = rpq.rpq_nfa_compile(rx, el.names)
        ref = plain(rpq, g, nfa, src, want_pairs, per_source)
        cap = ref.count + 3 if want_pairs else None
        qids.append(b.add(nfa, src, pairs_capacity=cap, per_source=per_source))
        expect.append(ref)
    for r in range(runs):
        say("batch run %d: %d queries, opts=%s" % (r, len(mix), opts))
        b.run()
        st = b.stats()
        assert st["n_queries"] == len(mix)
        if opts and opts.get("visit"):
            assert st["visit"] == opts["visit"]
        for qi, (rx, src, want_pairs, per_source), ref in zip(qids, mix, expect):
            got = b.result(qi)
            assert (got.count, got.hash, got.product_edges) == (ref.count, ref.hash, ref.product_edges), rx
            if want_pairs:
                assert np.array_equal(keys(got.pairs), keys(ref.pairs)), rx
            if per_source:
                assert np.array_equal(got.per_source.cpu().numpy(), ref.per_source.cpu().numpy()), rx
        # eager work between graph replays (a replay must not depend on leftovers)
        if og is not None and r == 0:
            rx, src, want_pairs, per_source = mix[0]
            want = oracle.rpq(og, rx, sources=src)
            assert expect[0].count == want.count and expect[0].hash == want.hash
    b.close()
    return expect


def test_batch_uniform_mix_matches_plain(rpq):
    el = synth.workload_graph("uniform_v1000_e5000_l4")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    og = oracle.OracleGraph.from_edgelist(el)
    rng = np.random.default_rng(5)
    mix = build_mix(rng, el.names, el.n_vertices, 24)
    for opts in (dict(batch_width=64, slots=3), dict(batch_width=128, slots=7, chunk_edges=5),
                 dict(batch_width=512, slots=2), dict(batch_width=64, slots=40),
                 dict(batch_width=128, slots=5, visit=rpq.RPQ_VISIT_SEEN_OR),
                 dict(batch_width=64, slots=40, chunk_edges=3, visit=rpq.RPQ_VISIT_SEEN_OR)):
        check_batch(rpq, g, el, mix, opts, og=og, runs=3)
    g.close()


def test_batch_against_oracle_random_graphs(rpq):
    rng = np.random.default_rng(99)
    names = ["a", "b", "c", "d"]
    for trial in range(12):
        n = int(rng.integers(2, 150))
        m = int(rng.integers(0, 5 * n))
        L = int(rng.integers(1, 5))
        src = rng.integers(0, n, size=m).astype(np.uint32)
        dst = rng.integers(0, n, size=m).astype(np.uint32)
        lab = rng.integers(0, L, size=m).astype(np.uint8)
        g = rpq.rpq_graph_create(src, lab, dst, n, L, names=names[:L])
        og = oracle.OracleGraph(n, src, lab, dst, L, names[:L])
        b = rpq.rpq_batch_create(g, dict(batch_width=int(rng.choice([64, 128, 256])),
                                          slots=int(rng.integers(1, 6)), chunk_edges=int(rng.integers(1, 70)),
                                          visit=1 + trial % 2))
        qs = []
        for i in range(int(rng.integers(1, 8))):
            rx = synth.random_regex(rng, names[:L])
            sources = synth.sample_sources(n, int(rng.integers(1, n + 1)), seed=trial * 100 + i)
            want = oracle.rpq(og, rx, sources=sources)
            nfa = rpq.rpq_nfa_compile(rx, names[:L])
            qs.append((b.add(nfa, sources, pairs_capacity=want.count + 1, per_source=True), want, rx))
        say("case: batch oracle trial=%d n=%d m=%d queries=%d" % (trial, n, m, len(qs)))
        b.run()
        for qid, want, rx in qs:
            got = b.result(qid)
            assert got.count == want.count, rx
            assert got.hash == want.hash, rx
            assert got.product_edges == want.product_edges, rx
            assert np.array_equal(keys(got.pairs), want.pairs), rx
            assert np.array_equal(got.per_source.cpu().numpy().view(np.uint64), want.per_source), rx
        b.close()
        g.close()


def test_batch_rmat18_mixed_sizes(rpq):
    el = synth.workload_graph("rmat18_l8")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    rng = np.random.default_rng(18)
    mix = []
    for i in range(16):
        rx = synth.random_regex(rng, el.names)   # 2..12 states
        if i % 2 == 0:
            mix.append((rx, np.array([int(rng.integers(0, el.n_vertices))], np.uint32), True, False))
        else:
            lo = int(rng.integers(0, el.n_vertices - 2048))
            mix.append((rx, np.arange(lo, lo + 2048, dtype=np.uint32), False, True))
    check_batch(rpq, g, el, mix, dict(batch_width=512, slots=8), runs=2)
    # one slot reused by every unit in turn: a retired unit's visited rows must be cleared
    # completely before the next unit seeds (regression: the clear raced with the slot reset)
    check_batch(rpq, g, el, mix, dict(batch_width=512, slots=1), runs=3)
    # the seen-OR scheme (expansion ORs new bits into the visited rows), against the plain two-read
    # results, with slots reused: a retired unit's visited rows are cleared from its first-visit log
    check_batch(rpq, g, el, mix, dict(batch_width=512, slots=8, visit=rpq.RPQ_VISIT_SEEN_OR), runs=2)
    check_batch(rpq, g, el, mix, dict(batch_width=512, slots=1, visit=rpq.RPQ_VISIT_SEEN_OR), runs=2)
    g.close()


def test_batch_invalid_sources_and_overflow(rpq):
    import torch
    el = synth.workload_graph("uniform_v1000_e5000_l4")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    nfa = rpq.rpq_nfa_compile("a.b*", el.names)
    b = rpq.rpq_batch_create(g, dict(batch_width=64, slots=2))
    b.add(nfa, np.array([5, 3], np.uint32))
    with pytest.raises(rpq.RpqError) as ei:
        b.run()
    assert ei.value.code == rpq.RPQ_EINVAL
    b.close()
    ref = rpq.rpq_eval(g, nfa, None, pairs=True)
    b = rpq.rpq_batch_create(g, dict(batch_width=64, slots=4))
    q = b.add(nfa, None, pairs_capacity=max(1, ref.count // 2))
    b.run()
    got = b.result(q)
    assert got.status == rpq.RPQ_EOVERFLOW and got.count == ref.count
    b.close()
    g.close()


def test_batch_autotune_then_run_matches_plain_and_oracle(rpq):
    """rpq_batch_autotune times candidate plans on a prefix of the queue; the plan it keeps must give
    every query exactly its plain result, and the oracle's for the single-source ones."""
    el = synth.workload_graph("rmat18_l8")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    og = oracle.OracleGraph.from_edgelist(el)
    rng = np.random.default_rng(2718)
    mix = build_mix(rng, el.names, el.n_vertices, 24)
    b = rpq.rpq_batch_create(g)
    qids, refs = [], []
    for rx, src, want_pairs, per_source in mix:
        nfa = rpq.rpq_nfa_compile(rx, el.names)
        ref = plain(rpq, g, nfa, src, want_pairs, per_source)
        refs.append(ref)
        qids.append(b.add(nfa, src, pairs_capacity=ref.count + 1 if want_pairs else None, per_source=per_source))
    say("case: autotune 24 queries on rmat18")
    tuned = b.autotune()
    say("tuned plan", tuned)
    assert tuned["batch_width"] in (64, 256, 512, 1024, 2048)
    b.run()
    for qi, (rx, src, want_pairs, per_source), ref in zip(qids, mix, refs):
        got = b.result(qi)
        assert (got.count, got.hash, got.product_edges) == (ref.count, ref.hash, ref.product_edges), rx
        if want_pairs:
            assert np.array_equal(keys(got.pairs), keys(ref.pairs)), rx
        if per_source:
            assert np.array_equal(got.per_source.cpu().numpy(), ref.per_source.cpu().numpy()), rx
        if src.size == 1:
            want = oracle.rpq(og, rx, sources=src)
            assert (got.count, got.hash, got.product_edges) == (want.count, want.hash, want.product_edges), rx
            assert np.array_equal(keys(got.pairs), want.pairs), rx
    b.close()
    g.close()


def test_batch_tiny_lists_defer_rows_without_changing_results(rpq):
    """With frontier lists, slice buffers and first-visit logs sized for 1/64 of the worst case, rows
    that do not fit wait for a later iteration (and overflowing logs clear their slot whole): every
    result must stay the plain one.  A length-bounded query needs exact depths and refuses the setting."""
    el = synth.workload_graph("rmat18_l8")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    rng = np.random.default_rng(64)
    mix = []
    for i in range(12):
        rx = ["a*", "a.b*", "(a|b).c*", "(a.b)*"][i % 4] if i < 4 else synth.random_regex(rng, el.names)
        if i % 3 == 0:
            mix.append((rx, np.array([int(rng.integers(0, el.n_vertices))], np.uint32), True, False))
        else:
            lo = int(rng.integers(0, el.n_vertices - 1024))
            mix.append((rx, np.arange(lo, lo + 1024, dtype=np.uint32), False, True))
    check_batch(rpq, g, el, mix, dict(batch_width=256, slots=6, list_share=64), runs=2)
    check_batch(rpq, g, el, mix, dict(batch_width=256, slots=6, list_share=64, visit=rpq.RPQ_VISIT_SEEN_OR), runs=2)
    b = rpq.rpq_batch_create(g, dict(batch_width=64, slots=2, list_share=64))
    b.add(rpq.rpq_nfa_compile("a*", el.names), np.array([1, 2], np.uint32), max_length=3)
    with pytest.raises(rpq.RpqError) as e:
        b.run()
    assert e.value.code == rpq.RPQ_EINVAL
    b.close()
    g.close()
