"""CPU checks of the seeded input generators shared by the oracle, the tests and the benchmark:
the same seed gives the same bytes, streams are prefix-stable, and the graphs have the stated
shape (sizes, label distribution, distinct triples)."""
import numpy as np

import synth


def test_request_stream_is_prefix_stable():
    # the serving runs quote "the first 200 requests of the stream": a longer stream starts with them
    names = synth.label_names(8)
    short = synth.serve_requests(200, 262144, names, seed=1018)
    long = synth.serve_requests(1000, 262144, names, seed=1018)
    for a, b in zip(short, long[:200]):
        assert a[0] == b[0] and a[1] == b[1]
        if a[0] == "crpq":
            assert a[2] == b[2] and a[3] == b[3]
        else:
            assert np.array_equal(a[2], b[2])
    kinds = [r[0] for r in long]
    for k, share in (("rpq_single", 0.4), ("rpq_slice", 0.4), ("crpq", 0.2)):
        assert abs(kinds.count(k) / len(kinds) - share) < 0.06, k


def test_sources_and_arrivals_are_seeded():
    a = synth.sample_sources(1000, 100, seed=3)
    assert np.array_equal(a, synth.sample_sources(1000, 100, seed=3))
    assert a.dtype == np.uint32 and np.all(np.diff(a.astype(np.int64)) > 0) and a.max() < 1000
    t = synth.poisson_arrivals(50.0, 2000, seed=9)
    assert np.all(np.diff(t) >= 0)
    assert abs(2000 / t[-1] - 50.0) < 5.0


def test_uniform_workload_has_exactly_the_stated_distinct_triples():
    el = synth.workload_graph("uniform_v1000_e5000_l4")
    assert el.n_vertices == 1000 and el.n_labels == 4 and el.n_edges == 5000
    keys = (el.src.astype(np.int64) << 24) | (el.label.astype(np.int64) << 20) | el.dst.astype(np.int64)
    assert np.unique(keys).size == 5000


def test_rmat_labels_follow_zipf_and_ids_stay_in_range():
    el = synth.workload_graph("rmat18_l8")
    assert el.n_vertices == 1 << 18 and el.n_edges == 16 << 18
    assert int(el.src.max()) < el.n_vertices and int(el.dst.max()) < el.n_vertices
    share = np.bincount(el.label, minlength=8) / el.n_edges
    want = synth.zipf_probs(8, 1.1)
    assert np.all(np.abs(share - want) < 0.005)
    assert share[0] == share.max()   # label a is the most frequent
    again = synth.workload_graph("rmat18_l8")
    assert np.array_equal(el.src, again.src) and np.array_equal(el.dst, again.dst)
