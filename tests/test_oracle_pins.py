"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these compare the oracle with itself: each check uses an independent
route -- values printed in the paper, relational algebra with Boolean
Warshall closure, brute-force walk enumeration with Python's ``re`` as the
acceptor, published SplitMix64 outputs, or closed forms.
"""
import itertools
import re

import numpy as np
import pytest

import oracle
from oracle import OracleGraph, crpq, crpq_bruteforce, mix64, pair_set, rpq
from oracle.automata import glushkov, leaf_count, parse, reverse_tree, thompson, to_text

from golden_io import load_worked_example

import synth


# ------------------------------------------------------------------------------------------------
# helpers that do NOT use the oracle's search
# ------------------------------------------------------------------------------------------------

def bool_closure(R):
    """Transitive closure by Boolean Floyd-Warshall (the paper's related-work
    Boolean algebra route, Section 9)."""
    R = R.copy()
    n = R.shape[0]
    for k in range(n):
        R |= np.outer(R[:, k], R[k, :])
    return R


def algebra_eval(tree, mats, n):
    """Relational evaluation of a regex: labels are edge relations, '.' is
    composition, '|' union, '*' reflexive-transitive closure, '+' transitive
    closure, '?' union with the identity (algebra-based approach, Section 2.2)."""
    I = np.eye(n, dtype=bool)
    kind = tree[0]
    if kind == "lab":
        return mats[tree[1]].copy()
    if kind == "cat":
        A = algebra_eval(tree[1], mats, n)
        B = algebra_eval(tree[2], mats, n)
        return (A.astype(np.int64) @ B.astype(np.int64)) > 0
    if kind == "alt":
        return algebra_eval(tree[1], mats, n) | algebra_eval(tree[2], mats, n)
    A = algebra_eval(tree[1], mats, n)
    if kind == "star":
        return I | bool_closure(A)
    if kind == "plus":
        return bool_closure(A)
    if kind == "opt":
        return I | A
    raise ValueError(kind)


def label_mats(n, L, edges):
    mats = [np.zeros((n, n), dtype=bool) for _ in range(L)]
    for (s, l, d) in edges:
        mats[l][s, d] = True
    return mats


def rel_of(res):
    return pair_set(res)


def mat_to_set(M):
    xs, ys = np.nonzero(M)
    return set(zip(xs.tolist(), ys.tolist()))


def random_tree(rng, L, depth=0, max_depth=4):
    if depth >= max_depth or (depth > 0 and rng.random() < 0.35):
        return ("lab", int(rng.integers(0, L)))
    op = rng.choice(["cat", "alt", "star", "plus", "opt"], p=[0.35, 0.25, 0.2, 0.1, 0.1])
    if op in ("cat", "alt"):
        return (str(op), random_tree(rng, L, depth + 1, max_depth), random_tree(rng, L, depth + 1, max_depth))
    return (str(op), random_tree(rng, L, depth + 1, max_depth))


def random_graph(rng, n, m, L):
    src = rng.integers(0, n, size=m).astype(np.uint32)
    dst = rng.integers(0, n, size=m).astype(np.uint32)
    lab = rng.integers(0, L, size=m).astype(np.uint8)
    return src, lab, dst


def synth_to_binary(ast):
    """Convert a synth AST (n-ary cat/alt lists) to the binary tuples used here."""
    kind = ast[0]
    if kind == "lab":
        return ast
    if kind in ("cat", "alt"):
        kids = [synth_to_binary(c) for c in ast[1]]
        t = kids[0]
        for k in kids[1:]:
            t = (kind, t, k)
        return t
    return (kind, synth_to_binary(ast[1]))


NAMES = ["a", "b", "c", "d"]


# ------------------------------------------------------------------------------------------------
# checksum
# ------------------------------------------------------------------------------------------------

def test_mix64_matches_published_splitmix64_outputs():
    # The first three outputs of SplitMix64 seeded with 0 (Steele, Lea, Flood 2014);
    # mix64(x) is the output produced from state x.
    gamma = 0x9E3779B97F4A7C15
    assert mix64(0) == 0xE220A8397B1DCDAF
    assert mix64(gamma) == 0x6E789E6AA1B965F4
    assert mix64((2 * gamma) & 0xFFFFFFFFFFFFFFFF) == 0x06C45D188009454F


def test_hash_keys_is_the_sum_of_the_published_outputs():
    # keys 0, gamma, 2*gamma give the three published outputs; their checksum is their sum mod 2^64,
    # whatever the order, and the empty sequence sums to 0
    from oracle import hash_keys
    gamma = 0x9E3779B97F4A7C15
    want = (0xE220A8397B1DCDAF + 0x6E789E6AA1B965F4 + 0x06C45D188009454F) & 0xFFFFFFFFFFFFFFFF
    keys = np.array([0, gamma, (2 * gamma) & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    assert hash_keys(keys) == want
    assert hash_keys(keys[::-1].copy()) == want
    assert hash_keys(np.zeros(0, dtype=np.uint64)) == 0
    assert hash_keys(np.array([5, 5], dtype=np.uint64)) == (2 * mix64(5)) & 0xFFFFFFFFFFFFFFFF


# ------------------------------------------------------------------------------------------------
# the paper's worked example (Section 1 footnote 1, Table 1, Sections 2.4, 3, 4)
# ------------------------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def wex():
    d = load_worked_example()
    g = OracleGraph(d["n"], d["src"], d["label"], d["dst"], len(d["names"]), d["names"], d["vertex_label"])
    return d, g


@pytest.mark.parametrize("automaton", ["glushkov", "thompson"])
def test_worked_example_abc_star_13_pairs(wex, automaton):
    d, g = wex
    res = rpq(g, d["query"], automaton=automaton)
    got = sorted((int(k) >> 32, int(k) & 0xFFFFFFFF) for k in res.pairs)
    assert got == d["pairs"]
    assert res.count == 13
    assert list(res.pairs) == sorted(res.pairs)


def test_worked_example_ab_block_AD(wex):
    # Section 2.4: the ab result block with source label A and destination label D
    # holds exactly {(v0, v10), (v0, v12)}.
    d, g = wex
    res = rpq(g, "ab")
    A = set(np.nonzero(d["vertex_label"] == d["vertex_label_names"].index("A"))[0].tolist())
    D = set(np.nonzero(d["vertex_label"] == d["vertex_label_names"].index("D"))[0].tolist())
    block = {(s, t) for (s, t) in pair_set(res) if s in A and t in D}
    assert block == {(0, 10), (0, 12)}


def test_worked_example_cycle_mutually_reachable(wex):
    # Section 3, Challenge 3: c* over the 4-cycle v10 -> v11 -> v12 -> v13 -> v10
    # makes all four vertices mutually reachable.
    d, g = wex
    got = pair_set(rpq(g, "c*", sources=np.array([10, 11, 12, 13], np.uint32)))
    for x in range(10, 14):
        for y in range(10, 14):
            assert (x, y) in got


def test_worked_example_v0_v9_shortest_walk_is_4_hops(wex):
    # Section 3 and Section 4.2: (v0, v9) is reached by the 4-hop walk
    # v0 -> v3 -> v12 -> v13 -> v9 and by no shorter accepted walk.
    d, g = wex
    src = np.array([0], np.uint32)
    assert (0, 9) in pair_set(rpq(g, "a.b.c.c", sources=src))
    shorter = pair_set(rpq(g, "a.b.c?", sources=src))
    assert (0, 9) not in shorter


def test_worked_example_witness_words(wex):
    # Footnote 1: (v2, v2), (v0, v7), (v0, v11) are witnessed by ab, abc, abccc.
    d, g = wex
    assert (2, 2) in pair_set(rpq(g, "ab"))
    assert (0, 7) in pair_set(rpq(g, "abc"))
    assert (0, 11) in pair_set(rpq(g, "abccc"))


def test_worked_example_crpq_q2(wex):
    # Section 1: Q2 on (u2, u3, u4) maps to {(v10,v0,v10), (v10,v0,v12), (v12,v0,v10),
    # (v12,v0,v12)}.  The query figure is missing; the reading used is
    # u3 -ab-> u2, u3 -ab-> u4, u2 -c*-> u4 with u3 labelled A and u2, u4 labelled D
    # (atoms from Section 2.4 and Section 6.2, labels from the GridMap block of S11).
    d, g = wex
    A = d["vertex_label_names"].index("A")
    D = d["vertex_label_names"].index("D")
    atoms = [(1, "ab", 0), (1, "ab", 2), (0, "c*", 2)]
    got = crpq(g, atoms, 3, var_label=[D, A, D])
    assert got == [(10, 0, 10), (10, 0, 12), (12, 0, 10), (12, 0, 12)]
    # the vertex-label condition of Definition 2 is what cuts the result to 4
    unlabelled = crpq(g, atoms, 3)
    assert set(got) < set(unlabelled)


# ------------------------------------------------------------------------------------------------
# closed forms: algebra-based evaluation with Boolean Warshall closure
# ------------------------------------------------------------------------------------------------

def test_star_is_reflexive_transitive_closure():
    rng = np.random.default_rng(7)
    for trial in range(20):
        n = int(rng.integers(1, 60))
        m = int(rng.integers(0, 3 * n + 1))
        src, lab, dst = random_graph(rng, n, m, 1)
        g = OracleGraph(n, src, lab, dst, 1, ["a"])
        A = label_mats(n, 1, zip(src.tolist(), lab.tolist(), dst.tolist()))[0]
        want = mat_to_set(np.eye(n, dtype=bool) | bool_closure(A))
        for automaton in ("glushkov", "thompson"):
            assert rel_of(rpq(g, "a*", automaton=automaton)) == want


def test_random_queries_match_relational_algebra():
    rng = np.random.default_rng(11)
    for trial in range(120):
        n = int(rng.integers(1, 25))
        m = int(rng.integers(0, 4 * n + 1))
        L = int(rng.integers(1, 5))
        src, lab, dst = random_graph(rng, n, m, L)
        g = OracleGraph(n, src, lab, dst, L, NAMES[:L])
        tree = random_tree(rng, L)
        want = mat_to_set(algebra_eval(tree, label_mats(n, L, zip(src.tolist(), lab.tolist(), dst.tolist())), n))
        text = to_text(tree, NAMES[:L])
        for automaton in ("glushkov", "thompson"):
            got = rel_of(rpq(g, text, automaton=automaton))
            assert got == want, (text, automaton)


def test_generator_strings_parse_with_the_printed_precedence():
    # the query strings drawn for the batched workload print '.' and '|' with
    # minimal parentheses; the oracle must read them with that precedence
    rng = np.random.default_rng(5)
    for trial in range(60):
        n = int(rng.integers(2, 20))
        L = 4
        src, lab, dst = random_graph(rng, n, 3 * n, L)
        g = OracleGraph(n, src, lab, dst, L, NAMES)
        ast = synth.random_regex_ast(rng, L, max_depth=4, zipf_s=1.1)
        text = synth.render_regex(ast, NAMES)
        want = mat_to_set(algebra_eval(synth_to_binary(ast), label_mats(n, L, zip(src.tolist(), lab.tolist(), dst.tolist())), n))
        assert rel_of(rpq(g, text)) == want, text


def test_composition_and_union_laws():
    rng = np.random.default_rng(3)
    for trial in range(30):
        n = int(rng.integers(2, 30))
        src, lab, dst = random_graph(rng, n, 3 * n, 3)
        g = OracleGraph(n, src, lab, dst, 3, NAMES[:3])
        t1, t2 = random_tree(rng, 3, max_depth=2), random_tree(rng, 3, max_depth=2)
        r1 = rel_of(rpq(g, to_text(t1, NAMES)))
        r2 = rel_of(rpq(g, to_text(t2, NAMES)))
        comp = {(x, z) for (x, y) in r1 for (y2, z) in r2 if y == y2}
        assert rel_of(rpq(g, "(%s).(%s)" % (to_text(t1, NAMES), to_text(t2, NAMES)))) == comp
        assert rel_of(rpq(g, "(%s)|(%s)" % (to_text(t1, NAMES), to_text(t2, NAMES)))) == r1 | r2
        ident = {(v, v) for v in range(n)}
        assert rel_of(rpq(g, "(%s)?" % to_text(t1, NAMES))) == r1 | ident


# ------------------------------------------------------------------------------------------------
# brute force on tiny graphs: every walk, Python's re as the acceptor
# ------------------------------------------------------------------------------------------------

def brute_force(n, edges, text, n_states, max_len=None):
    """All walks of length <= n * n_states - 1 (a shortest accepting product
    walk never repeats a (vertex, state) pair), or of length <= max_len when
    given, label words tested with re.fullmatch after mapping labels to
    letters."""
    pat = re.compile(text.replace(".", ""))
    out = set()
    by_src = {}
    for (s, l, d) in edges:
        by_src.setdefault(s, []).append((l, d))
    bound = n * n_states - 1 if max_len is None else max_len
    for s in range(n):
        frontier = {(s, "")}
        seen_all = set(frontier)
        for length in range(bound + 1):
            for (v, word) in frontier:
                if pat.fullmatch(word):
                    out.add((s, v))
            if length == bound:
                break
            nxt = set()
            for (v, word) in frontier:
                for (l, d) in by_src.get(v, ()):
                    item = (d, word + NAMES[l])
                    nxt.add(item)
            frontier = nxt
            if not frontier:
                break
    return out


def test_brute_force_tiny_graphs():
    rng = np.random.default_rng(2024)
    checked = 0
    while checked < 150:
        n = int(rng.integers(1, 5))
        m = int(rng.integers(0, 8))
        L = int(rng.integers(1, 4))
        src, lab, dst = random_graph(rng, n, m, L)
        tree = random_tree(rng, L, max_depth=3)
        q = leaf_count(tree) + 1
        if q > 4:
            continue
        edges = set(zip(src.tolist(), lab.tolist(), dst.tolist()))
        text = to_text(tree, NAMES[:L])
        g = OracleGraph(n, src, lab, dst, L, NAMES[:L])
        want = brute_force(n, edges, text, q)
        for automaton in ("glushkov", "thompson"):
            assert rel_of(rpq(g, text, automaton=automaton)) == want, text
        checked += 1


# ------------------------------------------------------------------------------------------------
# automata: acceptors agree with Python's re; Glushkov size
# ------------------------------------------------------------------------------------------------

def test_automata_accept_the_same_words_as_python_re():
    rng = np.random.default_rng(99)
    for trial in range(200):
        tree = random_tree(rng, 3)
        text = to_text(tree, NAMES[:3])
        pat = re.compile(text.replace(".", ""))
        gl, th = glushkov(tree), thompson(tree)
        assert gl.n_states == leaf_count(tree) + 1
        for _ in range(30):
            k = int(rng.integers(0, 7))
            word = [int(x) for x in rng.integers(0, 3, size=k)]
            want = bool(pat.fullmatch("".join(NAMES[w] for w in word)))
            assert gl.accepts(word) == want, (text, word)
            assert th.accepts(word) == want, (text, word)


def test_glushkov_state_count_for_abc_star_is_4():
    assert glushkov(parse("a.b.c*", NAMES)).n_states == 4


def test_parser_readings():
    # infix '|' alternation, postfix '+' one-or-more, '?' optional,
    # juxtaposition of single-letter labels is concatenation
    assert parse("abc*", NAMES) == parse("a.b.(c)*", NAMES)
    assert parse("a|b.c", NAMES) == ("alt", ("lab", 0), ("cat", ("lab", 1), ("lab", 2)))
    assert parse("a+", NAMES) == ("plus", ("lab", 0))
    assert parse("knows.knows*", ["knows", "hasTag"]) == ("cat", ("lab", 0), ("star", ("lab", 0)))
    # label names are matched longest first, so a name that extends another wins
    nm = ["a", "ab", "b"]
    assert parse("ab*", nm) == ("star", ("lab", 1))
    assert parse("a.b*", nm) == ("cat", ("lab", 0), ("star", ("lab", 2)))
    assert parse("aab", nm) == ("cat", ("lab", 0), ("lab", 1))
    with pytest.raises(ValueError):
        parse("a.(b", NAMES)
    with pytest.raises(ValueError):
        parse("x", NAMES)


# ------------------------------------------------------------------------------------------------
# invariants
# ------------------------------------------------------------------------------------------------

EQUIVALENT = [("(a|b)*", "(a*.b*)*"), ("(a.b)*.a", "a.(b.a)*"), ("(a*)*", "a*"),
              ("a.b*|a", "a.b*"), ("a+", "a.a*"), ("a?.a*", "a*"), ("(a|b).c", "a.c|b.c")]


@pytest.mark.parametrize("lhs,rhs", EQUIVALENT)
def test_regex_equivalences(lhs, rhs):
    rng = np.random.default_rng(abs(hash((lhs, rhs))) % (2 ** 32))
    for trial in range(10):
        n = int(rng.integers(1, 40))
        src, lab, dst = random_graph(rng, n, 3 * n, 3)
        g = OracleGraph(n, src, lab, dst, 3, NAMES[:3])
        assert rel_of(rpq(g, lhs)) == rel_of(rpq(g, rhs))


def test_transpose_invariant():
    # R_G(rho) reversed equals R_{G^T}(reverse(rho))
    rng = np.random.default_rng(17)
    for trial in range(40):
        n = int(rng.integers(1, 30))
        src, lab, dst = random_graph(rng, n, 3 * n, 3)
        g = OracleGraph(n, src, lab, dst, 3, NAMES[:3])
        gt = OracleGraph(n, dst, lab, src, 3, NAMES[:3])
        tree = random_tree(rng, 3)
        fwd = rel_of(rpq(g, to_text(tree, NAMES)))
        bwd = rel_of(rpq(gt, to_text(reverse_tree(tree), NAMES)))
        assert {(y, x) for (x, y) in fwd} == bwd


def test_monotone_in_edges():
    rng = np.random.default_rng(23)
    for trial in range(20):
        n = int(rng.integers(2, 30))
        src, lab, dst = random_graph(rng, n, 3 * n, 3)
        k = int(rng.integers(0, src.shape[0] + 1))
        g_small = OracleGraph(n, src[:k], lab[:k], dst[:k], 3, NAMES[:3])
        g_big = OracleGraph(n, src, lab, dst, 3, NAMES[:3])
        text = to_text(random_tree(rng, 3), NAMES)
        assert rel_of(rpq(g_small, text)) <= rel_of(rpq(g_big, text))


def test_duplicate_edges_change_nothing():
    rng = np.random.default_rng(29)
    n = 40
    src, lab, dst = random_graph(rng, n, 120, 3)
    g1 = OracleGraph(n, src, lab, dst, 3, NAMES[:3])
    g2 = OracleGraph(n, np.concatenate([src, src[:50]]), np.concatenate([lab, lab[:50]]),
                     np.concatenate([dst, dst[:50]]), 3, NAMES[:3])
    for text in ("a*", "a.b*.c", "(a|b).c*"):
        r1, r2 = rpq(g1, text), rpq(g2, text)
        assert np.array_equal(r1.pairs, r2.pairs)
        assert r1.product_edges == r2.product_edges
        assert r1.hash == r2.hash


def test_zero_length_walks_and_empty_inputs():
    # Definition 1 with a single-vertex path: (v, v) is in R(a*) for every
    # vertex, isolated ones included
    g = OracleGraph(5, np.array([0], np.uint32), np.array([0], np.uint8), np.array([1], np.uint32), 1, ["a"])
    assert rel_of(rpq(g, "a*")) == {(0, 0), (0, 1), (1, 1), (2, 2), (3, 3), (4, 4)}
    assert rel_of(rpq(g, "a+")) == {(0, 1)}
    r = rpq(g, "a*", sources=np.zeros(0, np.uint32))
    assert r.count == 0 and r.pairs.shape[0] == 0
    g0 = OracleGraph(3, np.zeros(0, np.uint32), np.zeros(0, np.uint8), np.zeros(0, np.uint32), 1, ["a"])
    assert rel_of(rpq(g0, "a")) == set()
    assert rel_of(rpq(g0, "a?")) == {(0, 0), (1, 1), (2, 2)}


# ------------------------------------------------------------------------------------------------
# product edges (the throughput numerator) in closed form
# ------------------------------------------------------------------------------------------------

def test_product_edges_closed_form_for_a_star():
    # Glushkov automaton of a*: state 0 (initial) and state 1 (the a position),
    # both with one a-transition to state 1.  From source s the reached pairs are
    # (s, 0) and (w, 1) for w in A+(s), so the examined product edges are
    # deg_a(s) + sum over w in A+(s) of deg_a(w).
    rng = np.random.default_rng(31)
    for trial in range(15):
        n = int(rng.integers(1, 50))
        src, lab, dst = random_graph(rng, n, 3 * n, 1)
        g = OracleGraph(n, src, lab, dst, 1, ["a"])
        A = label_mats(n, 1, zip(src.tolist(), lab.tolist(), dst.tolist()))[0]
        deg = A.sum(axis=1).astype(np.int64)
        Ap = bool_closure(A)
        want = int(sum(deg[s] + deg[Ap[s]].sum() for s in range(n)))
        assert rpq(g, "a*").product_edges == want


def test_product_edges_closed_form_for_a_dot_b():
    # Glushkov of a.b: states 0, 1 (a), 2 (b); 0 -a-> 1, 1 -b-> 2.  From s:
    # deg_a(s) + sum over a-successors w of deg_b(w).
    rng = np.random.default_rng(37)
    for trial in range(15):
        n = int(rng.integers(1, 50))
        src, lab, dst = random_graph(rng, n, 4 * n, 2)
        g = OracleGraph(n, src, lab, dst, 2, ["a", "b"])
        mats = label_mats(n, 2, zip(src.tolist(), lab.tolist(), dst.tolist()))
        da = mats[0].sum(axis=1).astype(np.int64)
        db = mats[1].sum(axis=1).astype(np.int64)
        want = int(sum(da[s] + db[mats[0][s]].sum() for s in range(n)))
        assert rpq(g, "a.b").product_edges == want


def test_hop_count_is_the_largest_first_reach_distance():
    # For a* the product pairs reached at depth k >= 1 are (w, 1) with w first
    # reached by a k-edge walk, so the deepest level is the largest such k over
    # the sources: found here from Boolean matrix powers, not by a search.
    n = 9
    path = OracleGraph(n, np.arange(n - 1, dtype=np.uint32), np.zeros(n - 1, np.uint8),
                       np.arange(1, n, dtype=np.uint32), 1, ["a"])
    assert rpq(path, "a*").max_hops == n - 1
    assert rpq(path, "a*", sources=np.array([5], np.uint32)).max_hops == n - 1 - 5
    rng = np.random.default_rng(41)
    for trial in range(15):
        n = int(rng.integers(1, 40))
        src, lab, dst = random_graph(rng, n, 2 * n, 1)
        g = OracleGraph(n, src, lab, dst, 1, ["a"])
        A = label_mats(n, 1, zip(src.tolist(), lab.tolist(), dst.tolist()))[0].astype(np.int64)
        seen = np.zeros((n, n), dtype=bool)
        P = np.eye(n, dtype=np.int64)
        ecc = np.zeros(n, dtype=np.int64)
        for k in range(1, n + 1):
            P = ((P @ A) > 0).astype(np.int64)
            new = (P > 0) & ~seen
            ecc[new.any(axis=1)] = k
            seen |= P > 0
        assert rpq(g, "a*").max_hops == int(ecc.max()), trial


# ------------------------------------------------------------------------------------------------
# per-source outputs and threading
# ------------------------------------------------------------------------------------------------

def test_per_source_and_threads_consistent():
    el = synth.uniform_graph(300, 1500, 4, seed=5)
    g = OracleGraph.from_edgelist(el)
    src = synth.sample_sources(300, 100, seed=6)
    r1 = rpq(g, "a.b*.c", sources=src)
    r4 = rpq(g, "a.b*.c", sources=src, threads=4)
    assert np.array_equal(r1.pairs, r4.pairs)
    assert np.array_equal(r1.per_source, r4.per_source)
    assert r1.product_edges == r4.product_edges
    keys = r1.pairs
    hs = [0] * len(src)
    cs = [0] * len(src)
    idx = {int(s): i for i, s in enumerate(src)}
    for k in keys.tolist():
        i = idx[k >> 32]
        cs[i] += 1
        hs[i] = (hs[i] + mix64(k)) & 0xFFFFFFFFFFFFFFFF
    assert [int(x) for x in r1.per_source[:, 0]] == cs
    assert [int(x) for x in r1.per_source[:, 1]] == hs
    assert r1.count == len(keys)


# ------------------------------------------------------------------------------------------------
# CRPQ join against brute force over all assignments
# ------------------------------------------------------------------------------------------------

def test_crpq_matches_bruteforce_tiny():
    rng = np.random.default_rng(41)
    for trial in range(40):
        n = int(rng.integers(1, 7))
        src, lab, dst = random_graph(rng, n, 2 * n + 2, 3)
        vl = rng.integers(0, 2, size=n).astype(np.uint8)
        g = OracleGraph(n, src, lab, dst, 3, NAMES[:3], vl)
        k = int(rng.integers(2, 4))
        n_atoms = int(rng.integers(1, 4))
        atoms = []
        for _ in range(n_atoms):
            x, y = int(rng.integers(0, k)), int(rng.integers(0, k))
            atoms.append((x, to_text(random_tree(rng, 3, max_depth=2), NAMES), y))
        var_label = [int(x) if rng.random() < 0.3 else None for x in rng.integers(0, 2, size=k)]
        binding = [None] * k
        if rng.random() < 0.3:
            binding[int(rng.integers(0, k))] = int(rng.integers(0, n))
        neq = [(0, 1)] if rng.random() < 0.3 else []
        got = crpq(g, atoms, k, binding=binding, var_label=var_label, neq=neq)
        want = crpq_bruteforce(g, atoms, k, binding=binding, var_label=var_label, neq=neq)
        assert got == want, (atoms, binding, var_label, neq)


def test_crpq_forward_matches_bruteforce_tiny():
    """The source-restricted join (atoms evaluated only from the values their source variable
    takes) against every assignment checked directly, on queries whose atoms point forward in
    the declared order: anchored chains, forks and triangles, self-loops, labels, inequalities."""
    rng = np.random.default_rng(43)
    shapes = [[(0, 1), (1, 2)], [(0, 1), (0, 1)], [(0, 1), (1, 2), (0, 2)], [(0, 1), (1, 1)],
              [(0, 0), (0, 1)], [(0, 2)]]
    for trial in range(60):
        n = int(rng.integers(1, 7))
        src, lab, dst = random_graph(rng, n, 2 * n + 3, 3)
        vl = rng.integers(0, 2, size=n).astype(np.uint8)
        g = OracleGraph(n, src, lab, dst, 3, NAMES[:3], vl)
        shape = shapes[trial % len(shapes)]
        k = 1 + max(max(x, y) for x, y in shape)
        atoms = [(x, to_text(random_tree(rng, 3, max_depth=2), NAMES), y) for x, y in shape]
        binding = [None] * k
        if rng.random() < 0.6:
            binding[0] = int(rng.integers(0, n))
        var_label = [int(x) if rng.random() < 0.25 else None for x in rng.integers(0, 2, size=k)]
        neq = [(0, k - 1)] if (k > 1 and rng.random() < 0.3) else []
        got = oracle.crpq_forward(g, atoms, k, binding=binding, var_label=var_label, neq=neq)
        want = crpq_bruteforce(g, atoms, k, binding=binding, var_label=var_label, neq=neq)
        assert got == want, (atoms, binding, var_label, neq)
    with pytest.raises(ValueError):
        oracle.crpq_forward(g, [(1, "a", 0)], 2)


# ------------------------------------------------------------------------------------------------
# length-bounded RPQs: only walks of at most k edges count (the extension the paper's conclusion
# names, enforced by the traversal depth)
# ------------------------------------------------------------------------------------------------

def test_length_bound_brute_force_tiny_graphs():
    rng = np.random.default_rng(2025)
    checked = 0
    while checked < 120:
        n = int(rng.integers(1, 5))
        m = int(rng.integers(0, 8))
        L = int(rng.integers(1, 4))
        src, lab, dst = random_graph(rng, n, m, L)
        tree = random_tree(rng, L, max_depth=3)
        q = leaf_count(tree) + 1
        if q > 4:
            continue
        edges = set(zip(src.tolist(), lab.tolist(), dst.tolist()))
        text = to_text(tree, NAMES[:L])
        g = OracleGraph(n, src, lab, dst, L, NAMES[:L])
        k = int(rng.integers(0, 6))
        want = brute_force(n, edges, text, q, max_len=k)
        for automaton in ("glushkov", "thompson"):
            r = rpq(g, text, automaton=automaton, max_length=k)
            assert rel_of(r) == want, (text, k)
            assert r.max_hops <= k
        checked += 1


def bounded_union_of_powers(M, lo, hi):
    """Union of the Boolean powers M^lo .. M^hi (empty when hi < lo)."""
    n = M.shape[0]
    Mi = M.astype(np.int64)
    P = np.eye(n, dtype=np.int64)
    for _ in range(lo):
        P = ((P @ Mi) > 0).astype(np.int64)
    out = np.zeros((n, n), dtype=bool)
    for _ in range(lo, hi + 1):
        out |= P > 0
        P = ((P @ Mi) > 0).astype(np.int64)
    return out


def compose(A, B):
    return (A.astype(np.int64) @ B.astype(np.int64)) > 0


def test_length_bound_closed_forms_by_matrix_powers():
    # R_k(a*) = A^0 | ... | A^k; R_k(a.b*) = A . (B^0 | ... | B^(k-1));
    # R_k((a.b)*) = union of (AB)^j for 2j <= k; R_k(a.b*.c) = A . (B^0 | ... | B^(k-2)) . C
    rng = np.random.default_rng(43)
    for trial in range(20):
        n = int(rng.integers(1, 30))
        src, lab, dst = random_graph(rng, n, 3 * n, 3)
        g = OracleGraph(n, src, lab, dst, 3, ["a", "b", "c"])
        A, B, C = label_mats(n, 3, zip(src.tolist(), lab.tolist(), dst.tolist()))
        AB = compose(A, B)
        for k in range(0, 7):
            forms = {
                "a*": bounded_union_of_powers(A, 0, k),
                "a.b*": compose(A, bounded_union_of_powers(B, 0, k - 1)),
                "(a.b)*": bounded_union_of_powers(AB, 0, k // 2),
                "a.b*.c": compose(compose(A, bounded_union_of_powers(B, 0, k - 2)), C),
            }
            for q, M in forms.items():
                assert rel_of(rpq(g, q, max_length=k)) == mat_to_set(M), (trial, q, k)


def test_length_bound_product_edges_closed_form_for_a_star():
    # Glushkov a*: (s, 0) at depth 0 and (w, 1) at w's first-reach distance d >= 1; a pair is
    # expanded (its a-edges examined) only when its depth is below k
    rng = np.random.default_rng(47)
    for trial in range(12):
        n = int(rng.integers(1, 40))
        src, lab, dst = random_graph(rng, n, 2 * n, 1)
        g = OracleGraph(n, src, lab, dst, 1, ["a"])
        A = label_mats(n, 1, zip(src.tolist(), lab.tolist(), dst.tolist()))[0]
        deg = A.sum(axis=1).astype(np.int64)
        # dist[s, w] = first d >= 1 with w in A^d(s), from Boolean powers
        dist = np.full((n, n), -1, dtype=np.int64)
        P = np.eye(n, dtype=np.int64)
        for d in range(1, n + 1):
            P = ((P @ A.astype(np.int64)) > 0).astype(np.int64)
            dist[(P > 0) & (dist < 0)] = d
        for k in (0, 1, 2, 3, 5):
            want = 0
            for s_ in range(n):
                if k >= 1:
                    want += int(deg[s_])
                    want += int(deg[(dist[s_] >= 1) & (dist[s_] <= k - 1)].sum())
            assert rpq(g, "a*", max_length=k).product_edges == want, (trial, k)


def test_length_bound_monotone_and_reaches_the_unbounded_result():
    el = synth.uniform_graph(200, 700, 3, seed=8)
    g = OracleGraph.from_edgelist(el)
    for q in ("a.b*", "(a|b).c*", "(a.b)*", "a?.c"):
        full = rpq(g, q)
        prev = set()
        for k in range(0, full.max_hops + 2):
            r = rpq(g, q, max_length=k)
            cur = rel_of(r)
            assert prev <= cur, (q, k)
            prev = cur
        assert cur == rel_of(full)
        # the pairs are complete at the deepest level; its pairs are expanded (their edges examined,
        # finding nothing new) only when the bound lies beyond it
        at = rpq(g, q, max_length=full.max_hops)
        assert (at.count, at.hash) == (full.count, full.hash)
        assert at.product_edges <= full.product_edges
        big = rpq(g, q, max_length=full.max_hops + 1)
        assert (big.count, big.hash, big.product_edges) == (full.count, full.hash, full.product_edges)
        # zero-length walks only at k = 0: (s, s) for every s exactly when the empty word is accepted
        z = rel_of(rpq(g, q, max_length=0))
        nullable = re.fullmatch(q.replace(".", ""), "") is not None
        assert z == ({(v, v) for v in range(200)} if nullable else set())
