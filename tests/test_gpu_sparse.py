"""GPU tests of RPQ_SPARSE (the per-source hash-set search): identical results to the oracle
and to the bit-parallel form, including per-source tallies, product edges and reverse walks."""
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


def test_sparse_against_oracle_random_graphs(rpq):
    rng = np.random.default_rng(77)
    names = ["a", "b", "c", "d"]
    for trial in range(25):
        n = int(rng.integers(1, 120))
        m = int(rng.integers(0, 5 * n))
        L = int(rng.integers(1, 5))
        src = rng.integers(0, n, size=m).astype(np.uint32)
        dst = rng.integers(0, n, size=m).astype(np.uint32)
        lab = rng.integers(0, L, size=m).astype(np.uint8)
        g = rpq.rpq_graph_create(src, lab, dst, n, L, flags=rpq.RPQ_BUILD_IN_CSR, names=names[:L])
        og = oracle.OracleGraph(n, src, lab, dst, L, names[:L])
        rx = synth.random_regex(rng, names[:L])
        sources = synth.sample_sources(n, int(rng.integers(1, n + 1)), seed=trial)
        say("case: sparse oracle trial=%d n=%d m=%d rx=%s" % (trial, n, m, rx))
        want = oracle.rpq(og, rx, sources=sources)
        nfa = rpq.rpq_nfa_compile(rx, names[:L])
        got = rpq.rpq_eval(g, nfa, sources, flags=rpq.RPQ_SPARSE, pairs=True, per_source=True)
        assert (got.count, got.hash, got.product_edges) == (want.count, want.hash, want.product_edges), rx
        assert np.array_equal(keys(got.pairs), want.pairs), rx
        assert np.array_equal(got.per_source.cpu().numpy().view(np.uint64), want.per_source), rx
        # reverse walks: the same answers as the dense form's reverse walks
        dense = rpq.rpq_eval(g, nfa, sources, flags=rpq.RPQ_REVERSE, pairs=True)
        sp = rpq.rpq_eval(g, nfa, sources, flags=rpq.RPQ_REVERSE | rpq.RPQ_SPARSE, pairs=True)
        assert (sp.count, sp.hash, sp.product_edges) == (dense.count, dense.hash, dense.product_edges), rx
        assert np.array_equal(keys(sp.pairs), keys(dense.pairs)), rx
        g.close()


def test_sparse_matches_dense_on_rmat18(rpq):
    el = synth.workload_graph("rmat18_l8")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    src = synth.sample_sources(el.n_vertices, 48, seed=1800)
    for q in synth.WORKLOADS["rmat18_l8"]["queries"] + ["c.d*", "(e|f).g*.h"]:
        say("case: sparse vs dense rmat18 %s" % q)
        nfa = rpq.rpq_nfa_compile(q, el.names)
        d = rpq.rpq_eval(g, nfa, src, pairs=True, per_source=True)
        s = rpq.rpq_eval(g, nfa, src, flags=rpq.RPQ_SPARSE, pairs=True, per_source=True)
        assert (s.count, s.hash, s.product_edges) == (d.count, d.hash, d.product_edges), q
        assert np.array_equal(keys(s.pairs), keys(d.pairs)), q
        assert np.array_equal(s.per_source.cpu().numpy(), d.per_source.cpu().numpy()), q
    # one source, then the pair buffer in two slices (resume by offset)
    nfa = rpq.rpq_nfa_compile("a.b*", el.names)
    one = np.array([int(src[3])], np.uint32)
    full = rpq.rpq_eval(g, nfa, one, flags=rpq.RPQ_SPARSE, pairs=True)
    if full.count >= 2:
        import torch
        half = full.count // 2
        buf = torch.empty(half, dtype=torch.int64, device="cuda")
        a = rpq.rpq_eval(g, nfa, one, flags=rpq.RPQ_SPARSE, pairs=buf, allow_overflow=True)
        assert a.status == rpq.RPQ_EOVERFLOW and a.written == half
        rest = torch.empty(full.count - half, dtype=torch.int64, device="cuda")
        b = rpq.rpq_eval(g, nfa, one, flags=rpq.RPQ_SPARSE, pairs=rest, pair_offset=half)
        assert np.array_equal(np.concatenate([keys(a.pairs), keys(b.pairs)]), keys(full.pairs))
    g.close()


def test_sparse_edge_cases(rpq):
    # isolated vertices with a language holding the empty word; empty source set
    n = 6
    src = np.array([0, 1], np.uint32)
    dst = np.array([1, 2], np.uint32)
    lab = np.array([0, 0], np.uint8)
    g = rpq.rpq_graph_create(src, lab, dst, n, 1, names=["a"])
    og = oracle.OracleGraph(n, src, lab, dst, 1, ["a"])
    nfa = rpq.rpq_nfa_compile("a*", ["a"])
    got = rpq.rpq_eval(g, nfa, None, flags=rpq.RPQ_SPARSE, pairs=True)
    want = oracle.rpq(og, "a*")
    assert np.array_equal(keys(got.pairs), want.pairs) and got.count == 6 + 3
    e = rpq.rpq_eval(g, nfa, np.zeros(0, np.uint32), flags=rpq.RPQ_SPARSE)
    assert e.count == 0 and e.hash == 0
    with pytest.raises(rpq.RpqError) as ei:
        rpq.rpq_eval(g, nfa, np.array([3, 2], np.uint32), flags=rpq.RPQ_SPARSE)
    assert ei.value.code == rpq.RPQ_EINVAL
    g.close()


def test_sparse_workspace_grows(rpq):
    """A source set that reaches far more than the starting table makes the call ask for more
    workspace; the binding retries and the result equals the dense form's."""
    el = synth.workload_graph("rmat18_l8")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    nfa = rpq.rpq_nfa_compile("a*", el.names)
    src = synth.sample_sources(el.n_vertices, 64, seed=31)
    need = rpq.rpq_eval_workspace_size(g, nfa, len(src), rpq.RPQ_SPARSE)
    s = rpq.rpq_eval(g, nfa, src, flags=rpq.RPQ_SPARSE)   # first call on this graph: no cached workspace
    d = rpq.rpq_eval(g, nfa, src)
    assert (s.count, s.hash, s.product_edges) == (d.count, d.hash, d.product_edges)
    assert s.count > need // 20   # reached far more states than the starting table holds
    g.close()
