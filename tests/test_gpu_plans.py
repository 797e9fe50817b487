"""Split plans (rpq_eval_split: the loop-cache and start-in-the-middle plans of Section 2.3) against
the CPU oracle of the concatenated expression.

R(head . tail) is the composition of R(head) and R(tail) (walks split at the boundary), so the
plan's keys, count, checksum and per-source tallies must equal the oracle's result for the
expression "(head).(tail)" evaluated directly, whatever the split point."""
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


def check_split(rpq, g, og, head, tail, sources, names, opts=None):
    res, info = rpq.rpq_eval_split(g, rpq.rpq_nfa_compile(head, names), rpq.rpq_nfa_compile(tail, names), sources,
                                   opts=opts, pairs=True, per_source=True)
    want = oracle.rpq(og, "(%s).(%s)" % (head, tail), sources=sources)
    assert res.count == want.count, (head, tail, res.count, want.count)
    assert res.hash == want.hash, (head, tail)
    got = res.pairs.cpu().numpy().view(np.uint64) if res.pairs is not None else np.zeros(0, np.uint64)
    assert np.array_equal(got, want.pairs), (head, tail)
    assert np.array_equal(res.per_source.cpu().numpy().view(np.uint64), want.per_source), (head, tail)
    return res, info, want


def test_split_random_graphs_and_split_points(rpq):
    rng = np.random.default_rng(2603)
    names = ["a", "b", "c", "d"]
    for trial in range(16):
        n = int(rng.integers(2, 300))
        m = int(rng.integers(0, 5 * n))
        src = rng.integers(0, n, size=m).astype(np.uint32)
        dst = rng.integers(0, n, size=m).astype(np.uint32)
        lab = rng.integers(0, 4, size=m).astype(np.uint8)
        g = rpq.rpq_graph_create(src, lab, dst, n, 4, names=names)
        og = oracle.OracleGraph(n, src, lab, dst, 4, names)
        sources = None if trial % 3 == 0 else synth.sample_sources(n, int(rng.integers(1, n + 1)), seed=trial)
        for _ in range(3):
            head = synth.random_regex(rng, names, max_leaves=4)
            tail = synth.random_regex(rng, names, max_leaves=4)
            say("case: split trial=%d n=%d m=%d head=%s tail=%s" % (trial, n, m, head, tail))
            check_split(rpq, g, og, head, tail, sources, names,
                        opts=dict(batch_width=int(rng.choice([64, 256])), visit=1 + trial % 2))
        g.close()


def test_split_special_cases(rpq):
    names = ["a", "b", "c"]
    # a path 0 -a-> 1 -b-> 2 -c-> 3 -c-> 4 and an isolated vertex 5
    src = np.array([0, 1, 2, 3], np.uint32)
    lab = np.array([0, 1, 2, 2], np.uint8)
    dst = np.array([1, 2, 3, 4], np.uint32)
    g = rpq.rpq_graph_create(src, lab, dst, 6, 3, names=names)
    og = oracle.OracleGraph(6, src, lab, dst, 3, names)
    say("case: split special cases")
    # the paper's worked query abc* split both ways: start in the middle (a | b.c*) and loop cache (a.b | c*)
    r1, i1, w1 = check_split(rpq, g, og, "a", "b.c*", None, names)
    r2, _, _ = check_split(rpq, g, og, "a.b", "c*", None, names)
    assert r1.count == r2.count == 3 and i1["middle_vertices"] == 1
    # zero-length walks on either side: (x, x) pairs of every source and self-loop lambda edges
    check_split(rpq, g, og, "a*", "b?", None, names)
    check_split(rpq, g, og, "c?", "c*", np.array([2, 3, 5], np.uint32), names)
    # a head that reaches nothing: no middle vertex, empty result
    r, info, _ = check_split(rpq, g, og, "b.a", "c*", None, names)
    assert r.count == 0 and info["middle_vertices"] == 0 and info["tail_pairs"] == 0
    g.close()


@pytest.fixture(scope="module")
def rmat18(rpq):
    el = synth.workload_graph("rmat18_l8")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    og = oracle.OracleGraph.from_edgelist(el)
    yield el, g, og
    g.close()


@pytest.mark.parametrize("head,tail", [("a", "b.c*"), ("a.b", "c*"), ("a", "b*.c"), ("(a|b)", "c*")])
def test_split_rmat18_sampled_sources(rpq, rmat18, head, tail):
    el, g, og = rmat18
    src = synth.sample_sources(el.n_vertices, 1024, seed=2604)
    say("case: split rmat18 head=%s tail=%s from 1024 sources" % (head, tail))
    res, info, want = check_split(rpq, g, og, head, tail, src, el.names)
    # the same keys as the one-automaton plan on the concatenated expression
    plain = rpq.rpq_eval(g, rpq.rpq_nfa_compile("(%s).(%s)" % (head, tail), el.names), src)
    assert (plain.count, plain.hash) == (res.count, res.hash)
    assert info["tail_pairs"] > 0 and info["middle_vertices"] > 0
