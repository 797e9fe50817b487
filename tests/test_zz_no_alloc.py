"""rpq_eval_noalloc (the allocation-free variant of rpq_eval, working in the library's static
device scratch) against rpq_eval on the same inputs: count, checksum, product edges, depth,
sorted pairs and per-source tallies must be identical.  Each case makes two calls in a row,
the second with a smaller input, so the second call starts from the scratch the first one left.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def rpq():
    import torch
    import paper_2602_20748_amd as m
    assert torch.cuda.is_available()
    m.load_library()
    return m


def both(rpq, g, nfa, src, **kw):
    """The same evaluation through rpq_eval and rpq_eval_noalloc, with caller-owned outputs."""
    import torch
    n = g.info()["n_vertices"] if src is None else len(src)
    ref = rpq.rpq_eval(g, nfa, src, pairs=True, per_source=True, **kw)
    pairs = torch.full((max(ref.count, 1),), -1, dtype=torch.int64, device="cuda")
    per_source = torch.full((n, 2), -1, dtype=torch.int64, device="cuda")
    got = rpq.rpq_eval_noalloc(g, nfa, src, pairs=pairs, per_source=per_source, **kw)
    torch.cuda.synchronize()
    return ref, got


def assert_same(ref, got):
    # levels counts the rounds of every group of units, so it depends on the plan (the scratch
    # may hold fewer units at once); every result field must be identical
    assert (got.count, got.hash, got.product_edges, got.max_depth, got.written) == \
        (ref.count, ref.hash, ref.product_edges, ref.max_depth, ref.written)
    assert np.array_equal(got.pairs.cpu().numpy(), ref.pairs.cpu().numpy())
    assert np.array_equal(got.per_source.cpu().numpy(), ref.per_source.cpu().numpy())


def test_noalloc_matches_rpq_eval_uniform_two_calls(rpq):
    el = synth.workload_graph("uniform_v1000_e5000_l4")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    say("case: noalloc uniform a.b.c* all-pairs")
    ref, got = both(rpq, g, rpq.rpq_nfa_compile("a.b.c*", el.names), None)
    assert ref.count > 0
    assert_same(ref, got)
    say("case: noalloc uniform (a|b)*.d from 37 sources")
    src = synth.sample_sources(el.n_vertices, 37, seed=5)
    ref, got = both(rpq, g, rpq.rpq_nfa_compile("(a|b)*.d", el.names), src)
    assert_same(ref, got)
    g.close()


def test_noalloc_matches_rpq_eval_rmat18_two_calls(rpq):
    # 4,096 sources on R-MAT scale 18 take several groups of units in the scratch (the plan is
    # narrowed to fit), then a smaller call of 64 sources with another automaton
    el = synth.workload_graph("rmat18_l8")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    src = synth.sample_sources(el.n_vertices, 4096, seed=1818)
    nfa = rpq.rpq_nfa_compile("a.b*.c", el.names)
    ws = rpq.rpq_eval_workspace_size(g, nfa, len(src), rpq.RPQ_PAIRS | rpq.RPQ_PER_SOURCE)
    say("case: noalloc rmat18 a.b*.c from 4096 sources (default workspace %d bytes)" % ws)
    assert ws > rpq.RPQ_NOALLOC_SCRATCH_BYTES   # so the narrowing is exercised
    ref, got = both(rpq, g, nfa, src)
    assert ref.count > 0
    assert_same(ref, got)
    say("case: noalloc rmat18 (a.b)* from 64 sources, length-bounded to 5")
    src2 = synth.sample_sources(el.n_vertices, 64, seed=1819)
    ref, got = both(rpq, g, rpq.rpq_nfa_compile("(a.b)*", el.names), src2, max_length=5)
    assert_same(ref, got)
    say("case: noalloc rmat18 a* from 64 sources")
    ref, got = both(rpq, g, rpq.rpq_nfa_compile("a*", el.names), src2)
    assert_same(ref, got)
    g.close()


def test_noalloc_rejects_what_does_not_fit(rpq):
    # host-side checks only: no kernel runs for either call
    el = synth.workload_graph("rmat18_l8")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    nfa = rpq.rpq_nfa_compile("a.b*", el.names)
    src = synth.sample_sources(el.n_vertices, 8192, seed=7)
    say("case: noalloc rejection of a fixed plan beyond the scratch")
    with pytest.raises(rpq.RpqError) as e:
        rpq.rpq_eval_noalloc(g, nfa, src, opts=dict(batch_width=4096, concurrency=2))
    assert e.value.code == rpq.RPQ_ENOMEM
    assert "scratch" in str(e.value)
    say("case: noalloc rejection of the sparse search")
    with pytest.raises(rpq.RpqError) as e:
        rpq.rpq_eval_noalloc(g, nfa, src[:1], flags=rpq.RPQ_SPARSE)
    assert e.value.code == rpq.RPQ_EUNSUPPORTED
    g.close()
