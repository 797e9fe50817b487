"""The batched mixed workload on R-MAT scale 22 (4,194,304 vertices, 16 labels Zipf(1.1)): 256
generated queries, even ones single-source from a random vertex, odd ones all-pairs over a
4,096-source slice.  The batched form (one persistent kernel in one captured graph launch) must
equal the plain form exactly; the plain form is checked against the oracle on every
single-source query and on 8 sampled sources of every slice query."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

N_QUERIES = 256
QUERY_SEED = 22 + 1000
SAMPLE_SEED = 22 + 2000


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
def w22(rpq):
    say("generating R-MAT scale 22")
    el = synth.workload_graph("rmat22_l16")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    mix = synth.rmat_query_mix(N_QUERIES, el.n_vertices, el.names, seed=QUERY_SEED)
    plain = []
    for i, (rx, src) in enumerate(mix):
        if i % 32 == 0:
            say("plain query %d / %d" % (i, N_QUERIES))
        nfa = rpq.rpq_nfa_compile(rx, el.names)
        if len(src) == 1:
            r = rpq.rpq_eval(g, nfa, src, pairs=True)
            plain.append(dict(count=r.count, hash=r.hash, eprod=r.product_edges,
                              pairs=r.pairs.cpu().numpy().view(np.uint64).copy()))
        else:
            r = rpq.rpq_eval(g, nfa, src, per_source=True)
            plain.append(dict(count=r.count, hash=r.hash, eprod=r.product_edges,
                              per_source=r.per_source.cpu().numpy().view(np.uint64).copy()))
    yield el, g, mix, plain
    g.close()


def test_batched_equals_plain(rpq, w22):
    el, g, mix, plain = w22
    b = rpq.rpq_batch_create(g)
    qids = []
    for (rx, src), p in zip(mix, plain):
        nfa = rpq.rpq_nfa_compile(rx, el.names)
        if len(src) == 1:
            qids.append(b.add(nfa, src, pairs_capacity=p["count"] + 1))
        else:
            qids.append(b.add(nfa, src, per_source=True))
    for run in range(2):   # the second run replays the captured graph
        say("batched run %d" % run)
        b.run()
        st = b.stats()
        say("batched: %d units, %d slots of width %d, %d iterations, %.1f ms" % (
            st["n_units"], st["slots"], st["batch_width"], st["iterations"], st["last_run_ms"]))
        for qi, (rx, src), p in zip(qids, mix, plain):
            r = b.result(qi)
            assert (r.count, r.hash, r.product_edges) == (p["count"], p["hash"], p["eprod"]), rx
            if len(src) == 1:
                assert np.array_equal(r.pairs.cpu().numpy().view(np.uint64), p["pairs"]), rx
            else:
                assert np.array_equal(r.per_source.cpu().numpy().view(np.uint64), p["per_source"]), rx
    b.close()


def test_plain_against_oracle_samples(rpq, w22):
    el, g, mix, plain = w22
    say("building the oracle graph")
    og = oracle.OracleGraph.from_edgelist(el)
    rng = np.random.default_rng(SAMPLE_SEED)
    tasks = []
    for i, ((rx, src), p) in enumerate(zip(mix, plain)):
        if len(src) == 1:
            tasks.append((i, rx, src, None))
        else:
            pos = np.sort(rng.choice(len(src), size=8, replace=False))
            tasks.append((i, rx, src[pos], pos))

    def check(t):
        i, rx, src, pos = t
        want = oracle.rpq(og, rx, sources=src, pairs=pos is None)
        p = plain[i]
        if pos is None:
            ok = (want.count, want.hash, want.product_edges) == (p["count"], p["hash"], p["eprod"]) and \
                np.array_equal(want.pairs, p["pairs"])
        else:
            ok = np.array_equal(want.per_source, p["per_source"][pos])
        return i, rx, ok

    bad = []
    with ThreadPoolExecutor(max_workers=16) as ex:
        for n_done, (i, rx, ok) in enumerate(ex.map(check, tasks)):
            if not ok:
                bad.append((i, rx))
            if n_done % 32 == 0:
                say("oracle checks: %d / %d" % (n_done, len(tasks)))
    assert not bad, bad
