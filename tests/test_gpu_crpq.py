"""GPU tests of crpq_eval (Definition 2): the join of atom results against the oracle's join,
the paper's worked example, closed forms on the typed social graph, and every traversal
strategy of the atoms."""
import sys

import numpy as np
import pytest

import oracle
import synth
from golden_io import load_worked_example
from social_forms import chain_hash, cycle_tuples, knows_components, reply_depth

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


def strategies(rpq):
    return [0, rpq.CRPQ_FORCE_DENSE, rpq.CRPQ_FORCE_SPARSE, rpq.CRPQ_NO_EDGE_SCAN | rpq.CRPQ_NO_REVERSE,
            rpq.CRPQ_FORCE_SPARSE | rpq.CRPQ_NO_EDGE_SCAN,
            # atoms in the batched persistent form (those that run forward, bit-parallel)
            rpq.CRPQ_BATCH_ATOMS, rpq.CRPQ_BATCH_ATOMS | rpq.CRPQ_FORCE_DENSE | rpq.CRPQ_NO_REVERSE | rpq.CRPQ_NO_EDGE_SCAN]


def rows(r):
    if r.tuples is None:
        return None
    t = r.tuples.cpu().numpy().view(np.uint32)
    return [tuple(int(v) for v in row) for row in t]


def test_worked_example_q2(rpq):
    d = load_worked_example()
    g = rpq.rpq_graph_create(d["src"], d["label"], d["dst"], d["n"], len(d["names"]), vertex_label=d["vertex_label"],
                             flags=rpq.RPQ_BUILD_IN_CSR, names=d["names"])
    A = d["vertex_label_names"].index("A")
    D = d["vertex_label_names"].index("D")
    atoms = [(1, "ab", 0), (1, "ab", 2), (0, "c*", 2)]
    want = [(10, 0, 10), (10, 0, 12), (12, 0, 10), (12, 0, 12)]
    for fl in strategies(rpq):
        say("case: worked example Q2 flags=%d" % fl)
        r = rpq.crpq_eval(g, atoms, 3, vertex_label=[D, A, D], tuples=True, flags=fl)
        assert rows(r) == want
        assert r.count == 4 and r.hash == oracle.crpq_hash(want)
        c = rpq.crpq_eval(g, atoms, 3, vertex_label=[D, A, D], flags=fl)   # count and checksum only
        assert (c.count, c.hash) == (4, r.hash)
    g.close()


def random_case(rng, n, names, n_vlabels):
    k = int(rng.integers(1, 5))
    # every variable in at least one atom: a random spanning chain plus extra atoms
    perm = rng.permutation(k)
    atoms = []
    for i in range(1, k):
        a, b = int(perm[i - 1]), int(perm[i])
        if rng.random() < 0.5:
            a, b = b, a
        atoms.append((a, synth.random_regex(rng, names, max_depth=3, max_leaves=5), b))
    for _ in range(int(rng.integers(0 if k > 1 else 1, 3))):
        atoms.append((int(rng.integers(0, k)), synth.random_regex(rng, names, max_depth=3, max_leaves=5),
                      int(rng.integers(0, k))))
    binding = [None] * k
    if rng.random() < 0.3:
        binding[int(rng.integers(0, k))] = int(rng.integers(0, n))
    var_label = [int(rng.integers(0, n_vlabels)) if rng.random() < 0.3 else None for _ in range(k)]
    domain = [None] * k
    if rng.random() < 0.3:
        i = int(rng.integers(0, k))
        domain[i] = rng.choice(n, size=int(rng.integers(1, n + 1)), replace=False).astype(np.uint32)
    neq = []
    if k >= 2 and rng.random() < 0.4:
        a, b = rng.choice(k, size=2, replace=False)
        neq.append((int(a), int(b)))
    return k, atoms, binding, var_label, domain, neq


def test_random_queries_against_oracle(rpq):
    rng = np.random.default_rng(2024)
    names = ["a", "b", "c"]
    for trial in range(30):
        n = int(rng.integers(2, 28))
        m = int(rng.integers(0, 4 * n))
        src = rng.integers(0, n, size=m).astype(np.uint32)
        dst = rng.integers(0, n, size=m).astype(np.uint32)
        lab = rng.integers(0, 3, size=m).astype(np.uint8)
        vl = rng.integers(0, 2, size=n).astype(np.uint8)
        g = rpq.rpq_graph_create(src, lab, dst, n, 3, vertex_label=vl, flags=rpq.RPQ_BUILD_IN_CSR, names=names)
        og = oracle.OracleGraph(n, src, lab, dst, 3, names, vl)
        for q in range(3):
            k, atoms, binding, var_label, domain, neq = random_case(rng, n, names, 2)
            want = oracle.crpq(og, atoms, k, binding=binding, var_label=var_label, neq=neq, var_domain=domain)
            wh = oracle.crpq_hash(want) if want and len(want[0]) else 0
            for fl in strategies(rpq):
                say("case: crpq random trial=%d q=%d n=%d atoms=%s binding=%s labels=%s neq=%s flags=%d"
                    % (trial, q, n, atoms, binding, var_label, neq, fl))
                r = rpq.crpq_eval(g, atoms, k, binding=binding, vertex_label=var_label, domain=domain, neq=neq,
                                  tuples=True, flags=fl)
                assert r.count == len(want)
                if r.n_free:
                    assert rows(r) == want
                    assert r.hash == wh
        g.close()


def test_isolated_variable_and_constants(rpq):
    """A variable in no atom is a cartesian factor; a query whose variables are all bound
    is a yes/no question (count 1 or 0)."""
    rng = np.random.default_rng(7)
    n = 9
    src = rng.integers(0, n, size=20).astype(np.uint32)
    dst = rng.integers(0, n, size=20).astype(np.uint32)
    lab = rng.integers(0, 2, size=20).astype(np.uint8)
    g = rpq.rpq_graph_create(src, lab, dst, n, 2, flags=rpq.RPQ_BUILD_IN_CSR, names=["a", "b"])
    og = oracle.OracleGraph(n, src, lab, dst, 2, ["a", "b"])
    atoms = [(0, "a.b*", 1)]
    want = oracle.crpq(og, atoms, 3)
    r = rpq.crpq_eval(g, atoms, 3, tuples=True)
    assert rows(r) == want and r.count == len(want)
    pair = oracle.rpq(og, "a.b*").pairs
    if len(pair):
        x, y = int(pair[0] >> np.uint64(32)), int(pair[0] & np.uint64(0xFFFFFFFF))
        r = rpq.crpq_eval(g, atoms, 2, binding=[x, y], tuples=True)
        assert r.count == 1 and r.n_free == 0
    g.close()


def test_workspace_grows_on_demand(rpq):
    """A workspace too small for the atoms makes the library ask for more (RPQ_ENOMEM with
    workspace_needed); the binding retries and the result is unchanged."""
    el = synth.workload_graph("uniform_v1000_e5000_l4")
    og = oracle.OracleGraph.from_edgelist(el)
    atoms = [(0, "a.b*", 1), (1, "c*", 2)]
    dom = [np.arange(0, 40, dtype=np.uint32), None, None]
    want = oracle.crpq(og, atoms, 3, var_domain=dom)
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, flags=rpq.RPQ_BUILD_IN_CSR,
                             names=el.names)
    r = rpq.crpq_eval(g, atoms, 3, domain=dom, tuples=True, workspace_bytes=1 << 16)
    assert rows(r) == want and r.hash == oracle.crpq_hash(want)
    g.close()


def test_hash_set_search_over_many_sources_hands_over_to_bit_parallel(rpq):
    # 150 directed a-cycles of 500 vertices: from every vertex, a* reaches its whole cycle.  x ranges
    # over 70,000 vertices, more than the bit-parallel search takes by source count, so the hash-set
    # search is tried first; at 500 reached vertices per source (above V/256) it passes its table cap
    # and the atom is evaluated bit-parallel instead.  Closed form: each source pairs with its cycle.
    n_cyc, L = 150, 500
    V = n_cyc * L
    v = np.arange(V, dtype=np.uint32)
    nxt = ((v // L) * L + (v % L + 1) % L).astype(np.uint32)
    g = rpq.rpq_graph_create(v, np.zeros(V, np.uint8), nxt, V, 1, names=["a"])
    dom = synth.sample_sources(V, 70000, seed=11)
    say("case: a* over 70,000 of 75,000 cycle vertices, auto / forced hash set / forced bit-parallel")
    auto = rpq.crpq_eval(g, [(0, "a*", 1)], 2, domain=[dom, None])
    assert auto.atom_strategy[0] == rpq.CRPQ_STRATEGY_DENSE
    forced = rpq.crpq_eval(g, [(0, "a*", 1)], 2, domain=[dom, None], flags=rpq.CRPQ_FORCE_SPARSE)
    assert forced.atom_strategy[0] == rpq.CRPQ_STRATEGY_SPARSE
    dense = rpq.crpq_eval(g, [(0, "a*", 1)], 2, domain=[dom, None], flags=rpq.CRPQ_FORCE_DENSE)
    xs = np.repeat(dom.astype(np.int64), L)
    ys = (((dom.astype(np.int64) // L) * L)[:, None] + np.arange(L)[None, :]).ravel()
    want = (xs.size, chain_hash(np.stack([xs, ys], axis=1)))
    for r in (auto, forced, dense):
        assert (r.count, r.hash) == want
    g.close()


def test_invalid_queries(rpq):
    el = synth.workload_graph("uniform_v1000_e5000_l4")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, names=el.names)
    with pytest.raises(rpq.RpqError) as e:
        rpq.crpq_eval(g, [(0, "a", 3)], 2)
    assert e.value.code == rpq.RPQ_EINVAL
    with pytest.raises(rpq.RpqError) as e:
        rpq.crpq_eval(g, [(0, "a", 1)], 2, binding=[None, el.n_vertices])
    assert e.value.code == rpq.RPQ_EINVAL
    with pytest.raises(rpq.RpqError) as e:   # vertex labels on a graph without them
        rpq.crpq_eval(g, [(0, "a", 1)], 2, vertex_label=[0, None])
    assert e.value.code == rpq.RPQ_EINVAL
    with pytest.raises(rpq.RpqError) as e:
        rpq.crpq_eval(g, [(0, "a", 1)], 2, domain=[np.array([5, el.n_vertices], np.uint32), None])
    assert e.value.code == rpq.RPQ_EINVAL
    # a variable that must differ from itself: empty result
    r = rpq.crpq_eval(g, [(0, "a", 1)], 2, neq=[(1, 1)])
    assert r.count == 0
    g.close()


# ------------------------------------------------------------------------------------------------
# typed social graph (persons, messages, tags)
# ------------------------------------------------------------------------------------------------
PERSON, MESSAGE, TAG = 0, 1, 2


def social_queries(rpq, el, P, M, sample_small, check_oracle_m=None):
    names = el.names
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, vertex_label=el.vertex_label,
                             flags=rpq.RPQ_BUILD_IN_CSR, names=names)
    tag1 = P + M
    # Query 1: messages with the top tag, their creator and every message up their reply chain
    q1_atoms = [(0, "hasTag", 1), (0, "hasCreator", 2), (0, "replyOf*", 3)]
    q1 = dict(binding=[None, tag1, None, None], vertex_label=[MESSAGE, TAG, PERSON, MESSAGE])
    say("case: social Q1 V=%d" % el.n_vertices)
    r1 = rpq.crpq_eval(g, q1_atoms, 4, tuples=True, **q1)
    t1 = r1.tuples.cpu().numpy().view(np.uint32).astype(np.int64)
    assert r1.n_free == 3 and t1.shape == (r1.count, 3)
    # closed form of the count: one creator per message, depth + 1 messages on its reply chain
    tagged = np.unique(el.src[(el.label == 3) & (el.dst == tag1)].astype(np.int64))
    depth = reply_depth(el, P, M)
    assert r1.count == int((depth[tagged - P] + 1).sum())
    assert np.array_equal(np.unique(t1[:, 0]), tagged)
    order = np.lexsort((t1[:, 2], t1[:, 1], t1[:, 0]))
    assert np.array_equal(order, np.arange(len(t1)))   # sorted lexicographically
    assert r1.hash == chain_hash(t1)
    c1 = rpq.crpq_eval(g, q1_atoms, 4, **q1)
    assert (c1.count, c1.hash) == (r1.count, r1.hash)
    if check_oracle_m is not None:
        og = check_oracle_m["og"]
        ms = check_oracle_m["m_sample"]
        want = oracle.crpq(og, q1_atoms, 4, binding=q1["binding"], var_label=q1["vertex_label"],
                           var_domain=[ms, None, None, None], threads=16)
        keep = np.isin(t1[:, 0], ms)
        assert [tuple(int(v) for v in row) for row in t1[keep]] == want
    # Query 2: a 3-cycle of knows.knows* over a person sample
    comp, deg = knows_components(el, P)
    cyc = [(0, "knows.knows*", 1), (1, "knows.knows*", 2), (2, "knows.knows*", 0)]
    want2 = cycle_tuples(sample_small, comp, deg)
    say("case: social Q2 sample=%d" % len(sample_small))
    dom = [sample_small] * 3
    r2 = rpq.crpq_eval(g, cyc, 3, domain=dom, vertex_label=[PERSON] * 3, tuples=True)
    assert r2.count == len(want2)
    assert np.array_equal(r2.tuples.cpu().numpy().view(np.uint32).astype(np.int64), want2)
    assert r2.hash == chain_hash(want2)
    return g, cyc, comp, deg


def test_social_graph_small(rpq):
    P, M, T = 4000, 40000, 512
    el = synth.social_graph(n_persons=P, n_messages=M, n_tags=T, knows_mean_degree=6.0, seed=4)
    og = oracle.OracleGraph.from_edgelist(el)
    rng = np.random.default_rng(4002)
    sample = np.sort(rng.choice(P, size=24, replace=False)).astype(np.uint32)
    tagged = np.unique(el.src[(el.label == 3) & (el.dst == P + M)])
    g, cyc, comp, deg = social_queries(rpq, el, P, M, sample,
                                       check_oracle_m=dict(og=og, m_sample=tagged[::5].astype(np.uint32)))
    # the same cycle under every atom strategy, and against the oracle's join
    want = oracle.crpq(og, cyc, 3, var_domain=[sample] * 3, var_label=[PERSON] * 3, threads=16)
    for fl in strategies(rpq):
        r = rpq.crpq_eval(g, cyc, 3, domain=[sample] * 3, vertex_label=[PERSON] * 3, tuples=True, flags=fl)
        assert rows(r) == want
    g.close()


@pytest.fixture(scope="module")
def social_full(rpq):
    say("generating the social graph (1M persons, 10M messages, 16,384 tags)")
    el = synth.social_graph()
    say("building the device graph")
    g = rpq.rpq_graph_create(el.src, el.label, el.dst, el.n_vertices, el.n_labels, vertex_label=el.vertex_label,
                             flags=rpq.RPQ_BUILD_IN_CSR, names=el.names)
    say("knows components")
    comp, deg = knows_components(el, 1_000_000)
    yield el, g, comp, deg
    g.close()


def test_social_full_size_query1(rpq, social_full):
    """Query 1 at full size: full count against the closed form, every tuple's checksum, and the
    oracle's join on a 1% sample of the tagged messages."""
    el, g, comp, deg = social_full
    P, M = 1_000_000, 10_000_000
    tag1 = P + M
    atoms = [(0, "hasTag", 1), (0, "hasCreator", 2), (0, "replyOf*", 3)]
    q1 = dict(binding=[None, tag1, None, None], vertex_label=[MESSAGE, TAG, PERSON, MESSAGE])
    say("case: social full Q1, count and checksum")
    c1 = rpq.crpq_eval(g, atoms, 4, **q1)
    say("  count %d, strategies %s, atom pairs %s" % (c1.count, c1.atom_strategy, c1.atom_pairs))
    tagged = np.unique(el.src[(el.label == 3) & (el.dst == tag1)].astype(np.int64))
    depth = reply_depth(el, P, M)
    assert c1.count == int((depth[tagged - P] + 1).sum())
    say("case: social full Q1, tuples")
    r1 = rpq.crpq_eval(g, atoms, 4, tuples=True, capacity=c1.count, **q1)
    t1 = r1.tuples.cpu().numpy().view(np.uint32).astype(np.int64)
    assert (r1.count, r1.hash) == (c1.count, c1.hash) and t1.shape == (c1.count, 3)
    assert np.array_equal(np.unique(t1[:, 0]), tagged)
    assert np.array_equal(np.lexsort((t1[:, 2], t1[:, 1], t1[:, 0])), np.arange(len(t1)))
    assert r1.hash == chain_hash(t1)
    rng = np.random.default_rng(4003)
    ms = np.sort(rng.choice(tagged, size=max(1, len(tagged) // 100), replace=False)).astype(np.uint32)
    say("building the oracle graph")
    og = oracle.OracleGraph.from_edgelist(el)
    say("oracle join on %d sampled messages" % len(ms))
    want = oracle.crpq(og, atoms, 4, binding=q1["binding"], var_label=q1["vertex_label"],
                       var_domain=[ms, None, None, None], threads=16)
    keep = np.isin(t1[:, 0], ms)
    assert [tuple(int(v) for v in row) for row in t1[keep]] == want


def test_social_full_size_cycle(rpq, social_full):
    """The 3-cycle of knows.knows* at full size: exact tuples over 128 persons, the sum of cubes
    for the count over 1,024."""
    el, g, comp, deg = social_full
    P = 1_000_000
    rng = np.random.default_rng(4004)
    cyc = [(0, "knows.knows*", 1), (1, "knows.knows*", 2), (2, "knows.knows*", 0)]
    s128 = np.sort(rng.choice(P, size=128, replace=False)).astype(np.uint32)
    say("case: social full 3-cycle, 128 persons, tuples")
    r = rpq.crpq_eval(g, cyc, 3, domain=[s128] * 3, vertex_label=[PERSON] * 3, tuples=True)
    want = cycle_tuples(s128, comp, deg)
    assert r.count == len(want)
    assert np.array_equal(r.tuples.cpu().numpy().view(np.uint32).astype(np.int64), want)
    assert r.hash == chain_hash(want)
    say("case: social full 3-cycle, 128 persons, atoms in the batched form")
    rb = rpq.crpq_eval(g, cyc, 3, domain=[s128] * 3, vertex_label=[PERSON] * 3, tuples=True,
                       flags=rpq.CRPQ_BATCH_ATOMS)
    assert all(st & rpq.CRPQ_STRATEGY_BATCHED for st in rb.atom_strategy[:3])
    assert rb.count == len(want) and rb.hash == r.hash
    assert np.array_equal(rb.tuples.cpu().numpy().view(np.uint32).astype(np.int64), want)
    s1024 = np.sort(rng.choice(P, size=1024, replace=False)).astype(np.uint32)
    say("case: social full 3-cycle, 1,024 persons, count only")
    r = rpq.crpq_eval(g, cyc, 3, domain=[s1024] * 3, vertex_label=[PERSON] * 3)
    live = s1024[deg[s1024] > 0]
    _, sizes = np.unique(comp[live], return_counts=True)
    say("  count %d (sum of cubes %d), join rows %d" % (r.count, int((sizes.astype(np.int64) ** 3).sum()),
                                                        r.join_rows))
    assert r.count == int((sizes.astype(np.int64) ** 3).sum())
