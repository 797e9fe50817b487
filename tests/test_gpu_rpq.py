"""GPU parity of the plain RPQ path against the CPU oracle (bit-exact).

Every test calls the HIP library through its C ABI (Python binding) and
compares keys, counts, checksums and product-edge counts with the oracle on
the same seeded inputs."""
import sys

import numpy as np
import pytest

import oracle
import synth
from golden_io import load_worked_example

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


def keys_np(res):
    return res.pairs.cpu().numpy().view(np.uint64) if res.pairs is not None else None


def gpu_graph(rpq, el, flags=0):
    return rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels,
                                vertex_label=getattr(el, "vertex_label", None), flags=flags, names=el.names)


def check_against_oracle(rpq, g, og, regex, sources=None, opts=None, names=None):
    names = names or og.names
    nfa = rpq.rpq_nfa_compile(regex, names)
    res = rpq.rpq_eval(g, nfa, sources, opts=opts, pairs=True, per_source=True)
    want = oracle.rpq(og, regex, sources=sources)
    got = keys_np(res)
    assert res.count == want.count, (regex, res.count, want.count)
    assert np.array_equal(got, want.pairs), regex
    assert res.hash == want.hash, regex
    assert res.product_edges == want.product_edges, (regex, res.product_edges, want.product_edges)
    ps = res.per_source.cpu().numpy().view(np.uint64)
    assert np.array_equal(ps, want.per_source), regex
    return res, want


def test_worked_example(rpq):
    d = load_worked_example()
    say("case: worked example abc*")
    g = rpq.rpq_graph_create(d["src"], d["label"], d["dst"], d["n"], len(d["names"]), names=d["names"])
    og = oracle.OracleGraph(d["n"], d["src"], d["label"], d["dst"], len(d["names"]), d["names"])
    res, _ = check_against_oracle(rpq, g, og, d["query"])
    got = sorted((int(k) >> 32, int(k) & 0xFFFFFFFF) for k in keys_np(res))
    assert got == d["pairs"]
    assert res.count == 13
    for q in ("ab", "c*", "a.b.c.c", "(a|b|c)*", "b.c+"):
        check_against_oracle(rpq, g, og, q)
    g.close()


def test_uniform_1000_all_pairs_full(rpq):
    say("case: uniform 1000/5000 a.b.c* all-pairs")
    el = synth.workload_graph("uniform_v1000_e5000_l4")
    g = gpu_graph(rpq, el)
    og = oracle.OracleGraph.from_edgelist(el)
    info = g.info()
    assert info["n_edges"] == og.n_edges == 5000
    res, want = check_against_oracle(rpq, g, og, "a.b.c*")
    assert res.count > 0
    g.close()


@pytest.mark.parametrize("width", [64, 128, 256, 512, 1024, 2048, 4096])
def test_batch_shapes_do_not_change_results(rpq, width):
    el = synth.workload_graph("uniform_v1000_e5000_l4")
    g = gpu_graph(rpq, el)
    og = oracle.OracleGraph.from_edgelist(el)
    src = synth.sample_sources(1000, 700, seed=3)
    for conc in (1, 3):
        for chunk in (1, 5, 64):
            say("case: uniform width=%d conc=%d chunk=%d" % (width, conc, chunk))
            check_against_oracle(rpq, g, og, "(a|b).c*.d?", sources=src,
                                 opts=dict(batch_width=width, concurrency=conc, chunk_edges=chunk, sync_every=1 + chunk % 3))
    g.close()


def test_random_small_graphs_and_queries(rpq):
    rng = np.random.default_rng(77)
    names = ["a", "b", "c", "d"]
    for trial in range(60):
        n = int(rng.integers(1, 200))
        m = int(rng.integers(0, 6 * n + 1))
        L = int(rng.integers(1, 5))
        src = rng.integers(0, n, size=m).astype(np.uint32)
        dst = rng.integers(0, n, size=m).astype(np.uint32)
        lab = rng.integers(0, L, size=m).astype(np.uint8)
        if m and rng.random() < 0.3:   # duplicated edges
            src, dst, lab = np.concatenate([src, src[: m // 2]]), np.concatenate([dst, dst[: m // 2]]), \
                np.concatenate([lab, lab[: m // 2]])
        regex = synth.random_regex(rng, names[:L])
        say("case: random trial=%d n=%d m=%d L=%d q=%s" % (trial, n, m, L, regex))
        g = rpq.rpq_graph_create(src, lab, dst, n, L, names=names[:L])
        og = oracle.OracleGraph(n, src, lab, dst, L, names[:L])
        sources = None if rng.random() < 0.5 else synth.sample_sources(n, int(rng.integers(1, n + 1)), seed=trial)
        width = int(rng.choice([64, 128, 256, 512, 1024, 2048, 4096]))
        # both visit schemes, alternating by trial
        check_against_oracle(rpq, g, og, regex, sources=sources,
                             opts=dict(batch_width=width, concurrency=int(rng.integers(1, 4)),
                                       chunk_edges=int(rng.integers(1, 100)), visit=1 + trial % 2))
        g.close()


@pytest.fixture(scope="module")
def rmat18(rpq):
    el = synth.workload_graph("rmat18_l8")
    g = gpu_graph(rpq, el)
    og = oracle.OracleGraph.from_edgelist(el)
    yield el, g, og
    g.close()


def test_rmat18_graph_ingest(rpq, rmat18):
    el, g, og = rmat18
    info = g.info()
    assert info["n_edges"] == og.n_edges
    assert info["n_edges_in"] == el.n_edges
    row_ptr, dst = rpq.rpq_graph_export_csr(g)
    rp = row_ptr.cpu().numpy().view(np.uint32).astype(np.int64)
    ds = dst.cpu().numpy().view(np.uint32)
    L = el.n_labels
    # the oracle's adjacency is sorted by (label, dst) per vertex: same order as the CSR rows
    off = og.off.astype(np.int64)
    assert rp[-1] == og.n_edges
    assert np.array_equal(rp[0:el.n_vertices * L:L], off[:-1])
    assert np.array_equal(ds, og.dst[: og.n_edges])
    labs = np.repeat(np.tile(np.arange(L), el.n_vertices), np.diff(rp))
    assert np.array_equal(labs, og.lab[: og.n_edges])


@pytest.mark.parametrize("regex", ["a*", "a.b*", "(a|b).c*", "a.b*.c", "(a.b)*"])
def test_rmat18_sampled_sources(rpq, rmat18, regex):
    el, g, og = rmat18
    src = synth.sample_sources(el.n_vertices, 1024, seed=2018)
    say("case: rmat18 sampled 1024 sources q=%s" % regex)
    check_against_oracle(rpq, g, og, regex, sources=src)


@pytest.mark.parametrize("regex", ["a*", "a.b*.c", "(a.b)*"])
@pytest.mark.parametrize("visit", ["two-reads", "seen-or"])
def test_rmat18_visit_schemes(rpq, rmat18, regex, visit):
    # each way of finding a target word's new bits, forced (the default at this size is two reads),
    # over eight 128-wide units advanced two at a time: pairs, per-source tallies and product
    # edges against the oracle
    el, g, og = rmat18
    src = synth.sample_sources(el.n_vertices, 1000, seed=2026)
    say("case: rmat18 visit=%s q=%s" % (visit, regex))
    v = rpq.RPQ_VISIT_TWO_READS if visit == "two-reads" else rpq.RPQ_VISIT_SEEN_OR
    check_against_oracle(rpq, g, og, regex, sources=src, opts=dict(visit=v, batch_width=128, concurrency=2))


@pytest.mark.parametrize("regex", ["a*", "a.b*", "(a|b).c*", "a.b*.c", "(a.b)*"])
def test_rmat18_all_pairs_per_source_at_samples(rpq, rmat18, regex):
    import torch
    el, g, og = rmat18
    say("case: rmat18 all-pairs per-source q=%s" % regex)
    nfa = rpq.rpq_nfa_compile(regex, el.names)
    res = rpq.rpq_eval(g, nfa, None, per_source=True)
    ps = res.per_source.cpu().numpy().view(np.uint64)
    assert int(ps[:, 0].sum(dtype=np.uint64)) == res.count
    assert int(ps[:, 1].sum(dtype=np.uint64)) == res.hash
    src = synth.sample_sources(el.n_vertices, 1024, seed=4242)
    want = oracle.rpq(og, regex, sources=src, pairs=False)
    assert np.array_equal(ps[src.astype(np.int64)], want.per_source)


def test_empty_and_single_sources(rpq):
    el = synth.workload_graph("uniform_v1000_e5000_l4")
    g = gpu_graph(rpq, el)
    og = oracle.OracleGraph.from_edgelist(el)
    nfa = rpq.rpq_nfa_compile("a*", el.names)
    r = rpq.rpq_eval(g, nfa, np.zeros(0, np.uint32), per_source=True)
    assert r.count == 0 and r.hash == 0
    for s in (0, 999, 517):
        check_against_oracle(rpq, g, og, "a*", sources=np.array([s], np.uint32))
        check_against_oracle(rpq, g, og, "b.a+", sources=np.array([s], np.uint32))
    g.close()


def test_isolated_vertices_and_zero_length_walks(rpq):
    # vertices 3..9 have no edges: a* still holds (v, v) for each (Definition 1)
    src = np.array([0, 1, 2], np.uint32)
    dst = np.array([1, 2, 0], np.uint32)
    lab = np.array([0, 0, 1], np.uint8)
    g = rpq.rpq_graph_create(src, lab, dst, 10, 2, names=["a", "b"])
    og = oracle.OracleGraph(10, src, lab, dst, 2, ["a", "b"])
    for q in ("a*", "a?", "b*", "(a|b)*", "a+", "a.b"):
        check_against_oracle(rpq, g, og, q)
    g.close()


def test_overflow_and_resume(rpq):
    import torch
    el = synth.workload_graph("uniform_v1000_e5000_l4")
    g = gpu_graph(rpq, el)
    og = oracle.OracleGraph.from_edgelist(el)
    nfa = rpq.rpq_nfa_compile("a.b.c*", el.names)
    want = oracle.rpq(og, "a.b.c*")
    cap = max(1, want.count // 3 + 7)
    got = []
    off = 0
    while True:
        buf = torch.empty(cap, dtype=torch.int64, device="cuda")
        r = rpq.rpq_eval(g, nfa, None, pairs=buf, pair_offset=off, allow_overflow=True)
        assert r.count == want.count
        got.append(r.pairs.cpu().numpy().view(np.uint64).copy())
        off += r.written
        if r.status == rpq.RPQ_OK:
            break
        assert r.status == rpq.RPQ_EOVERFLOW and r.written == cap
    assert np.array_equal(np.concatenate(got), want.pairs)
    g.close()


def test_largest_automaton_and_label_alphabet(rpq):
    # 64 edge labels (the most a graph may have) and queries of 31 label occurrences,
    # i.e. 32 automaton states (the most the device tables hold); one more occurrence is refused
    rng = np.random.default_rng(64)
    names = ["l%d" % i for i in range(64)]
    n, m = 300, 6000
    src = rng.integers(0, n, size=m).astype(np.uint32)
    dst = rng.integers(0, n, size=m).astype(np.uint32)
    lab = rng.integers(0, 64, size=m).astype(np.uint8)
    g = rpq.rpq_graph_create(src, lab, dst, n, 64, names=names)
    og = oracle.OracleGraph(n, src, lab, dst, 64, names)
    union31 = "(" + "|".join(names[:31]) + ")*"
    chain31 = "(%s).(%s)*.(%s)" % ("|".join(names[33:43]), "|".join(names[43:53]), "|".join(names[53:64]))
    for regex in (union31, chain31, "(" + "|".join(names[32:63]) + ")+"):
        say("case: 32-state query %s..." % regex[:40])
        assert rpq.rpq_nfa_compile(regex, names).n_states == 32
        for sources in (None, synth.sample_sources(n, 77, seed=5)):
            check_against_oracle(rpq, g, og, regex, sources=sources)
    with pytest.raises(rpq.RpqError) as ei:
        rpq.rpq_nfa_compile("(" + "|".join(names[:32]) + ")*", names)
    assert ei.value.code == rpq.RPQ_EUNSUPPORTED
    g.close()


def test_invalid_inputs(rpq):
    import torch
    el = synth.workload_graph("uniform_v1000_e5000_l4")
    g = gpu_graph(rpq, el)
    nfa = rpq.rpq_nfa_compile("a*", el.names)
    for bad in (np.array([5, 3], np.uint32), np.array([2, 2], np.uint32), np.array([1000], np.uint32)):
        with pytest.raises(rpq.RpqError) as ei:
            rpq.rpq_eval(g, nfa, bad)
        assert ei.value.code == rpq.RPQ_EINVAL
    tiny = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(rpq.RpqError) as ei:
        rpq.rpq_eval(g, nfa, np.array([1, 2], np.uint32), workspace=tiny)
    assert ei.value.code == rpq.RPQ_ENOMEM
    with pytest.raises(rpq.RpqError) as ei:
        rpq.rpq_eval(g, nfa, None, flags=rpq.RPQ_REVERSE)
    assert ei.value.code == rpq.RPQ_EUNSUPPORTED
    with pytest.raises(rpq.RpqError) as ei:
        rpq.rpq_eval(g, nfa, np.array([1], np.uint32), opts=dict(batch_width=96))
    assert ei.value.code == rpq.RPQ_EINVAL
    with pytest.raises(rpq.RpqError) as ei:
        rpq.rpq_eval(g, nfa, np.array([1], np.uint32), opts=dict(visit=3))
    assert ei.value.code == rpq.RPQ_EINVAL
    with pytest.raises(ValueError):
        rpq.rpq_eval(g, nfa, np.array([1], np.uint32), opts=dict(visits=2))
    big = rpq.rpq_nfa_compile("a", ["a", "b", "c", "d", "e"])
    big.delta[0 * 64 + 4] = 2
    with pytest.raises(rpq.RpqError) as ei:
        rpq.rpq_eval(g, big, np.array([1], np.uint32))
    assert ei.value.code == rpq.RPQ_EINVAL
    with pytest.raises(rpq.RpqError) as ei:
        rpq.rpq_graph_create(np.array([0], np.uint32), np.array([7], np.uint8), np.array([1], np.uint32), 5, 4)
    assert ei.value.code == rpq.RPQ_EINVAL
    with pytest.raises(rpq.RpqError) as ei:
        rpq.rpq_graph_create(np.array([0], np.uint32), np.array([0], np.uint8), np.array([5], np.uint32), 5, 4)
    assert ei.value.code == rpq.RPQ_EINVAL
    g.close()


def test_reverse_traversal_matches_transposed_graph(rpq):
    el = synth.workload_graph("uniform_v1000_e5000_l4")
    g = gpu_graph(rpq, el, flags=rpq.RPQ_BUILD_IN_CSR)
    ogt = oracle.OracleGraph(el.n_vertices, el.dst, el.label, el.src, el.n_labels, el.names)
    from oracle.automata import parse, reverse_tree, to_text
    for q in ("a.b.c*", "(a|b).c*.d", "a*"):
        say("case: reverse q=%s" % q)
        nfa = rpq.rpq_nfa_compile(q, el.names)
        src = synth.sample_sources(1000, 300, seed=9)
        res = rpq.rpq_eval(g, nfa, src, flags=rpq.RPQ_REVERSE, pairs=True)
        want = oracle.rpq(ogt, to_text(reverse_tree(parse(q, el.names)), el.names), sources=src)
        assert res.count == want.count
        assert np.array_equal(keys_np(res), want.pairs)
        assert res.hash == want.hash
    g.close()


def test_repeated_calls_are_deterministic(rpq, rmat18):
    el, g, og = rmat18
    nfa = rpq.rpq_nfa_compile("(a|b).c*", el.names)
    src = synth.sample_sources(el.n_vertices, 5000, seed=1)
    r1 = rpq.rpq_eval(g, nfa, src, per_source=True)
    r2 = rpq.rpq_eval(g, nfa, src, per_source=True, opts=dict(batch_width=128, concurrency=5, chunk_edges=7))
    assert (r1.count, r1.hash, r1.product_edges) == (r2.count, r2.hash, r2.product_edges)
    assert np.array_equal(r1.per_source.cpu().numpy(), r2.per_source.cpu().numpy())
