"""Streamed result pairs (rpq_eval_stream) against the CPU oracle.

The keys arrive chunk by chunk through a host callback while the traversal goes on (the
double-buffered drain of the unified result buffer, Section 6.1).  The concatenation of the chunks
must be the oracle's sorted distinct key sequence, with the same count and checksum; on the large
case, where the keys do not fit one device buffer, count and checksum are taken by the oracle's
checksum over every streamed key and compared with the count-only evaluation, and the pairs of
sampled sources are compared with the oracle's."""
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
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    yield el, g
    g.close()


@pytest.fixture(scope="module")
def og18(rmat18):
    return oracle.OracleGraph.from_edgelist(rmat18[0])


class Collect:
    """Sink that keeps every chunk (small results)."""

    def __init__(self):
        self.chunks = []

    def __call__(self, keys):
        self.chunks.append(keys.copy())

    def keys(self):
        return np.concatenate(self.chunks) if self.chunks else np.zeros(0, dtype=np.uint64)


def test_stream_uniform_all_pairs_small_chunks(rpq):
    el = synth.workload_graph("uniform_v1000_e5000_l4")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    og = oracle.OracleGraph.from_edgelist(el)
    for regex, chunk in (("a.b.c*", 997), ("(a|b)*.d", 4096), ("a.b.c*", 1)):
        say("case: stream uniform %s all-pairs, chunks of %d keys" % (regex, chunk))
        want = oracle.rpq(og, regex)
        sink = Collect()
        res = rpq.rpq_eval_stream(g, rpq.rpq_nfa_compile(regex, el.names), sink, chunk_keys=chunk, per_source=True)
        got = sink.keys()
        assert res.count == want.count == res.written == got.size
        assert np.array_equal(got, want.pairs), regex
        assert res.hash == want.hash == oracle.hash_keys(got)
        assert res.product_edges == want.product_edges
        assert np.array_equal(res.per_source.cpu().numpy().view(np.uint64), want.per_source)
        assert all(c.size <= chunk for c in sink.chunks)
    g.close()


def test_stream_many_groups_against_oracle(rpq, rmat18, og18):
    # narrow units, two at a time: 2,048 sources take four groups, so windows of one group are
    # drained while the next group's levels run; chunk size is prime (windows straddle sources)
    el, g = rmat18
    src = synth.sample_sources(el.n_vertices, 2048, seed=2602)
    for regex in ("a.b*.c", "(a|b).c*"):
        say("case: stream rmat18 %s from 2048 sources in 4 groups" % regex)
        want = oracle.rpq(og18, regex, sources=src, threads=16)
        sink = Collect()
        res = rpq.rpq_eval_stream(g, rpq.rpq_nfa_compile(regex, el.names), sink, sources=src,
                                  opts=dict(batch_width=256, concurrency=2), chunk_keys=100003, per_source=True)
        got = sink.keys()
        assert res.count == want.count == got.size
        assert np.array_equal(got, want.pairs), regex
        assert res.hash == want.hash
        assert np.array_equal(res.per_source.cpu().numpy().view(np.uint64), want.per_source)


def test_stream_astar_65536_sources_beyond_one_buffer(rpq, rmat18, og18):
    # a* from 65,536 sampled sources: billions of keys (tens of GB), streamed through two 64 MB
    # chunks; every key is checked for order and summed by the oracle's checksum
    el, g = rmat18
    src = synth.sample_sources(el.n_vertices, 65536, seed=1818)
    nfa = rpq.rpq_nfa_compile("a*", el.names)
    say("case: count-only a* from 65536 sources")
    ref = rpq.rpq_eval(g, nfa, src, per_source=True)
    picks = np.sort(np.random.default_rng(7).choice(src, 8, replace=False)).astype(np.uint64)
    state = dict(n=0, h=0, last=-1, chunks=0, picked=[[] for _ in picks])

    def sink(keys):
        if keys.size:
            assert int(keys[0]) > state["last"]
            assert keys.size == 1 or bool(np.all(keys[1:] > keys[:-1]))
            state["last"] = int(keys[-1])
        state["n"] += keys.size
        state["h"] = (state["h"] + oracle.hash_keys(keys)) & 0xFFFFFFFFFFFFFFFF
        state["chunks"] += 1
        srcs = keys >> np.uint64(32)
        lo = np.searchsorted(srcs, picks, side="left")
        hi = np.searchsorted(srcs, picks, side="right")
        for i in range(len(picks)):
            if hi[i] > lo[i]:
                state["picked"][i].append(keys[lo[i]:hi[i]].copy())

    say("case: streamed a* from 65536 sources, chunks of 8M keys")
    res = rpq.rpq_eval_stream(g, nfa, sink, sources=src, chunk_keys=1 << 23, per_source=True)
    say("streamed %d keys in %d chunks" % (state["n"], state["chunks"]))
    assert res.count == ref.count == state["n"] == res.written
    assert res.hash == ref.hash == state["h"]
    assert state["chunks"] > 2
    assert np.array_equal(res.per_source.cpu().numpy(), ref.per_source.cpu().numpy())
    want = oracle.rpq(og18, "a*", sources=picks.astype(np.uint32), threads=8)
    got = np.concatenate([np.concatenate(c) if c else np.zeros(0, np.uint64) for c in state["picked"]])
    assert np.array_equal(got, want.pairs)


def test_stream_cancel_and_errors(rpq, rmat18):
    el, g = rmat18
    src = synth.sample_sources(el.n_vertices, 4096, seed=3)
    nfa = rpq.rpq_nfa_compile("a*", el.names)
    seen = []

    def stop_after_three(keys):
        seen.append(keys.size)
        return len(seen) >= 3

    say("case: stream cancelled by the sink after three chunks")
    with pytest.raises(rpq.RpqError) as e:
        rpq.rpq_eval_stream(g, nfa, stop_after_three, sources=src, chunk_keys=50000)
    assert e.value.code == rpq.RPQ_ECANCELED
    assert seen == [50000, 50000, 50000]
    say("case: a full stream after the cancelled one")
    ref = rpq.rpq_eval(g, nfa, src)
    sink = Collect()
    res = rpq.rpq_eval_stream(g, nfa, sink, sources=src, chunk_keys=1 << 22)
    assert res.count == ref.count == sink.keys().size and res.hash == ref.hash
    say("case: stream argument errors (host checks only)")
    with pytest.raises(rpq.RpqError) as e:
        rpq.rpq_eval_stream(g, nfa, sink, sources=src, chunk_keys=0)
    assert e.value.code == rpq.RPQ_EINVAL
    with pytest.raises(rpq.RpqError) as e:
        rpq.rpq_eval_stream(g, nfa, sink, sources=src[:4], flags=rpq.RPQ_SPARSE)
    assert e.value.code == rpq.RPQ_EUNSUPPORTED
