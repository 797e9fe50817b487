"""Seeded synthetic inputs for regular path query evaluation.

This module only draws inputs: edge lists, query strings, source sets and
arrival times.  It holds none of the query-evaluation arithmetic, so both the
CPU oracle (``oracle/``) and the HIP library binding use it without sharing any
evaluation code.

Every generator takes an explicit integer seed and uses
``numpy.random.default_rng(seed)``; the same seed gives the same bytes.

Graphs are returned as raw edge lists (``src`` uint32, ``label`` uint8, ``dst``
uint32).  Generators that model multigraphs (R-MAT) may emit the same
(src, label, dst) triple more than once; evaluation treats the edge set as a
set, so both sides remove duplicates at ingest.

Workload shapes follow the paper's evaluation (Section 8.1): power-law graphs
with several edge labels standing in for LDBC SNB and StackOverflow, and the
query shapes of Table 2 (a*, a?b*, ab*, abcd, abc*, ab*c, (a1+...+ak)b*, ...).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "EdgeList", "label_names", "zipf_probs", "uniform_graph", "rmat_graph",
    "social_graph", "random_regex_ast", "render_regex", "random_regex",
    "regex_leaf_count", "sample_sources", "poisson_arrivals", "serve_requests", "WORKLOADS",
    "workload_graph", "rmat_query_mix",
]


@dataclasses.dataclass
class EdgeList:
    """A labelled directed edge list plus its vertex and label universe."""
    n_vertices: int
    n_labels: int
    src: np.ndarray          # uint32 [E]
    label: np.ndarray        # uint8  [E]
    dst: np.ndarray          # uint32 [E]
    names: List[str]         # edge-label names, index = label id
    vertex_label: Optional[np.ndarray] = None   # uint8 [V] or None
    vertex_label_names: Optional[List[str]] = None

    @property
    def n_edges(self) -> int:
        return int(self.src.shape[0])


def label_names(n_labels: int) -> List[str]:
    """Single-letter names a, b, c, ... for label ids 0..n_labels-1."""
    if n_labels > 26:
        return ["l%d" % i for i in range(n_labels)]
    return [chr(ord("a") + i) for i in range(n_labels)]


def zipf_probs(n: int, s: float) -> np.ndarray:
    """P(rank r) proportional to r^-s for r = 1..n; index 0 is rank 1."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-float(s))
    return w / w.sum()


def _draw_labels(rng: np.random.Generator, n: int, n_labels: int, zipf_s: Optional[float]) -> np.ndarray:
    if zipf_s is None:
        return rng.integers(0, n_labels, size=n, dtype=np.int64).astype(np.uint8)
    return rng.choice(n_labels, size=n, p=zipf_probs(n_labels, zipf_s)).astype(np.uint8)


def uniform_graph(n_vertices: int, n_edges: int, n_labels: int, seed: int) -> EdgeList:
    """Exactly ``n_edges`` distinct (src, label, dst) triples drawn uniformly.

    Self-loops are allowed.  Triples are kept in first-drawn order.
    """
    rng = np.random.default_rng(seed)
    total = n_vertices * n_vertices * n_labels
    if n_edges > total:
        raise ValueError("more distinct edges requested than exist")
    keys = np.empty(0, dtype=np.int64)
    while keys.shape[0] < n_edges:
        need = n_edges - keys.shape[0]
        draw = rng.integers(0, total, size=2 * need + 16, dtype=np.int64)
        allk = np.concatenate([keys, draw])
        _, first = np.unique(allk, return_index=True)
        keys = allk[np.sort(first)]
    keys = keys[:n_edges]
    src = (keys // (n_vertices * n_labels)).astype(np.uint32)
    rem = keys % (n_vertices * n_labels)
    lab = (rem // n_vertices).astype(np.uint8)
    dst = (rem % n_vertices).astype(np.uint32)
    return EdgeList(n_vertices, n_labels, src, lab, dst, label_names(n_labels))


def _threads() -> int:
    import os
    return max(1, min(16, os.cpu_count() or 1))


def _pcg64_at(state: dict, draws: int) -> np.random.Generator:
    """A generator whose PCG64 stream starts `draws` 64-bit outputs after `state`."""
    bg = np.random.PCG64()
    bg.state = state
    bg.advance(draws)
    return np.random.Generator(bg)


def rmat_graph(scale: int, edge_factor: int = 16, probs: Sequence[float] = (0.57, 0.19, 0.19, 0.05),
               n_labels: int = 8, zipf_s: float = 1.1, seed: int = 0,
               chunk: int = 1 << 22) -> EdgeList:
    """R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004) with Zipf edge labels.

    ``2**scale`` vertices, ``edge_factor * 2**scale`` drawn edges.  At each of
    the ``scale`` recursion levels a quadrant is picked with probabilities
    (a, b, c, d); the source bit is set for c and d, the destination bit for b
    and d.  Vertex ids are then relabelled by a seeded random permutation (as
    Graph500 does) so that id order carries no locality.  Labels are drawn
    Zipf(zipf_s) with label 0 the most frequent.  Duplicates are kept.

    The draws form one PCG64 stream of ``default_rng(seed)``: for each chunk of
    edges, one uniform double per edge and level (level-major within the
    chunk), then the permutation, then one uniform per edge for its label.
    Chunks are drawn on several threads, each from its own generator advanced
    to the chunk's position in that stream, so the bytes do not depend on the
    thread count.
    """
    from concurrent.futures import ThreadPoolExecutor
    rng = np.random.default_rng(seed)
    state0 = rng.bit_generator.state
    n = 1 << scale
    m = edge_factor * n
    cum = np.cumsum(np.asarray(probs, dtype=np.float64))
    cum[-1] = 1.0
    # quadrant = number of cumulative bounds <= u: c or d (>= 2) sets the source bit, b or d
    # (1 or 3) the destination bit
    c0, c1, c2 = cum[0], cum[1], cum[2]
    src = np.empty(m, dtype=np.uint32)
    dst = np.empty(m, dtype=np.uint32)

    def draw_chunk(lo: int) -> None:
        hi = min(m, lo + chunk)
        g = _pcg64_at(state0, lo * scale)
        u = np.empty(hi - lo, dtype=np.float64)
        s = np.zeros(hi - lo, dtype=np.uint32)
        d = np.zeros(hi - lo, dtype=np.uint32)
        for level in range(scale):
            g.random(out=u)
            shift = np.uint32(scale - 1 - level)
            sbit = u >= c1
            s |= sbit.astype(np.uint32) << shift
            d |= (((u >= c0) & ~sbit) | (u >= c2)).astype(np.uint32) << shift
        src[lo:hi] = s
        dst[lo:hi] = d

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(draw_chunk, range(0, m, chunk)))
    rng = _pcg64_at(state0, m * scale)
    perm = rng.permutation(n).astype(np.uint32)
    src = perm[src]
    dst = perm[dst]
    lab = np.empty(m, dtype=np.uint8)
    cdf = np.cumsum(zipf_probs(n_labels, zipf_s))
    cdf /= cdf[-1]
    state1 = rng.bit_generator.state

    def draw_labels(lo: int) -> None:
        # one uniform per edge, mapped through the Zipf CDF (what Generator.choice does with p=)
        hi = min(m, lo + chunk)
        u = _pcg64_at(state1, lo).random(hi - lo)
        lab[lo:hi] = np.searchsorted(cdf, u, side="right").astype(np.uint8)

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(draw_labels, range(0, m, chunk)))
    return EdgeList(n, n_labels, src, lab, dst, label_names(n_labels))


SOCIAL_LABELS = ["knows", "hasCreator", "replyOf", "hasTag"]
SOCIAL_VERTEX_LABELS = ["Person", "Message", "Tag"]


def social_graph(n_persons: int = 1_000_000, n_messages: int = 10_000_000, n_tags: int = 16_384,
                 knows_mean_degree: float = 20.0, knows_gamma: float = 2.5,
                 reply_p: float = 0.3, tag_zipf_s: float = 1.2, seed: int = 4) -> EdgeList:
    """Typed social graph shaped like the LDBC SNB schema used by the paper's CRPQs.

    Vertex ids: persons [0, P), messages [P, P+M), tags [P+M, P+M+T); the
    vertex label is the type (0 person, 1 message, 2 tag).  Edge labels:

    * knows (0): Chung-Lu power law with exponent ``knows_gamma`` and mean
      degree ``knows_mean_degree``; undirected, stored in both directions;
      self-pairs dropped.
    * hasCreator (1): every message points to one uniform person.
    * replyOf (2): message depth D = Geometric(reply_p) - 1 on {0, 1, ...};
      depth-0 messages are roots and a depth-d message points to a uniform
      message of depth d-1.  A message whose depth level has no parent
      candidates becomes a root.
    * hasTag (3): every message gets 1-3 distinct tags (count uniform), tags
      drawn Zipf(tag_zipf_s) with tag rank 1 at id P+M.
    """
    rng = np.random.default_rng(seed)
    P, M, T = n_persons, n_messages, n_tags
    V = P + M + T
    # knows: Chung-Lu with expected degree w_i proportional to i^(-1/(gamma-1))
    w = np.arange(1, P + 1, dtype=np.float64) ** (-1.0 / (knows_gamma - 1.0))
    w = w / w.sum()
    n_und = int(round(P * knows_mean_degree / 2.0))
    ku = rng.choice(P, size=n_und, p=w).astype(np.uint32)
    kv = rng.choice(P, size=n_und, p=w).astype(np.uint32)
    keep = ku != kv
    ku, kv = ku[keep], kv[keep]
    # relabel persons so that high-weight persons are spread over the id range
    pperm = rng.permutation(P).astype(np.uint32)
    ku, kv = pperm[ku], pperm[kv]
    k_src = np.concatenate([ku, kv])
    k_dst = np.concatenate([kv, ku])
    # hasCreator
    msg = np.arange(P, P + M, dtype=np.uint32)
    creator = rng.integers(0, P, size=M, dtype=np.int64).astype(np.uint32)
    # replyOf
    depth = rng.geometric(reply_p, size=M).astype(np.int64) - 1
    order = np.argsort(depth, kind="stable")
    sdepth = depth[order]
    max_d = int(sdepth[-1]) if M else 0
    starts = np.searchsorted(sdepth, np.arange(max_d + 2))
    r_src, r_dst = [], []
    for d in range(1, max_d + 1):
        lo, hi = starts[d], starts[d + 1]
        plo, phi = starts[d - 1], starts[d]
        if hi <= lo:
            continue
        if phi <= plo:
            continue       # no parent candidates: these messages stay roots
        child = order[lo:hi]
        parent = order[plo + rng.integers(0, phi - plo, size=hi - lo, dtype=np.int64)]
        r_src.append((P + child).astype(np.uint32))
        r_dst.append((P + parent).astype(np.uint32))
    r_src = np.concatenate(r_src) if r_src else np.empty(0, np.uint32)
    r_dst = np.concatenate(r_dst) if r_dst else np.empty(0, np.uint32)
    # hasTag: 1-3 distinct tags per message
    cnt = rng.integers(1, 4, size=M, dtype=np.int64)
    tp = zipf_probs(T, tag_zipf_s)
    tags = rng.choice(T, size=(M, 3), p=tp).astype(np.int64)
    for _ in range(64):
        bad1 = (tags[:, 1] == tags[:, 0]) & (cnt >= 2)
        bad2 = ((tags[:, 2] == tags[:, 0]) | (tags[:, 2] == tags[:, 1])) & (cnt >= 3)
        nb1, nb2 = int(bad1.sum()), int(bad2.sum())
        if nb1 == 0 and nb2 == 0:
            break
        if nb1:
            tags[bad1, 1] = rng.choice(T, size=nb1, p=tp)
        if nb2:
            tags[bad2, 2] = rng.choice(T, size=nb2, p=tp)
    t_src = np.concatenate([msg, msg[cnt >= 2], msg[cnt >= 3]])
    t_dst = np.concatenate([tags[:, 0], tags[cnt >= 2, 1], tags[cnt >= 3, 2]]).astype(np.uint32) + np.uint32(P + M)
    src = np.concatenate([k_src, msg, r_src, t_src]).astype(np.uint32)
    dst = np.concatenate([k_dst, creator, r_dst, t_dst]).astype(np.uint32)
    lab = np.concatenate([
        np.full(k_src.shape[0], 0, np.uint8), np.full(M, 1, np.uint8),
        np.full(r_src.shape[0], 2, np.uint8), np.full(t_src.shape[0], 3, np.uint8)])
    vl = np.concatenate([np.zeros(P, np.uint8), np.ones(M, np.uint8), np.full(T, 2, np.uint8)])
    return EdgeList(V, 4, src, lab, dst, list(SOCIAL_LABELS), vl, list(SOCIAL_VERTEX_LABELS))


# ----------------------------------------------------------------------------------------------
# query strings
# ----------------------------------------------------------------------------------------------
# An AST is a nested tuple: ("lab", i) | ("cat", [c...]) | ("alt", [c...]) | ("star", c)
# | ("plus", c) | ("opt", c).  It is only used to draw and print query strings.

def random_regex_ast(rng: np.random.Generator, n_labels: int, max_depth: int = 4,
                     zipf_s: Optional[float] = 1.1, leaf_p: float = 0.35):
    """One random regex AST of depth <= max_depth over labels 0..n_labels-1."""
    p = zipf_probs(n_labels, zipf_s) if zipf_s is not None else None

    def leaf():
        return ("lab", int(rng.choice(n_labels, p=p)) if p is not None else int(rng.integers(0, n_labels)))

    def gen(depth):
        if depth >= max_depth or (depth > 0 and rng.random() < leaf_p):
            return leaf()
        op = rng.choice(["cat", "alt", "star", "opt", "plus"], p=[0.4, 0.25, 0.2, 0.075, 0.075])
        if op in ("cat", "alt"):
            k = 2 if rng.random() < 0.75 else 3
            return (op, [gen(depth + 1) for _ in range(k)])
        return (op, gen(depth + 1))

    return gen(0)


def regex_leaf_count(ast) -> int:
    """Number of label occurrences in an AST."""
    kind = ast[0]
    if kind == "lab":
        return 1
    if kind in ("cat", "alt"):
        return sum(regex_leaf_count(c) for c in ast[1])
    return regex_leaf_count(ast[1])


def render_regex(ast, names: Sequence[str]) -> str:
    """Print an AST as a query string: '|' alternation, '.' concatenation,
    postfix '*', '+', '?', parentheses where precedence needs them."""
    def prec(a):
        return {"alt": 0, "cat": 1}.get(a[0], 2)

    def r(a):
        kind = a[0]
        if kind == "lab":
            return names[a[1]]
        if kind == "alt":
            return "|".join(r(c) for c in a[1])
        if kind == "cat":
            return ".".join("(" + r(c) + ")" if prec(c) < 1 else r(c) for c in a[1])
        op = {"star": "*", "plus": "+", "opt": "?"}[kind]
        inner = a[1]
        s = r(inner)
        if inner[0] != "lab":
            s = "(" + s + ")"
        return s + op

    return r(ast)


def random_regex(rng: np.random.Generator, names: Sequence[str], max_depth: int = 4,
                 min_leaves: int = 1, max_leaves: int = 11, zipf_s: Optional[float] = 1.1) -> str:
    """A query string whose label-occurrence count lies in [min_leaves, max_leaves]
    (redrawn until it does)."""
    for _ in range(10000):
        ast = random_regex_ast(rng, len(names), max_depth=max_depth, zipf_s=zipf_s)
        k = regex_leaf_count(ast)
        if min_leaves <= k <= max_leaves:
            return render_regex(ast, names)
    raise RuntimeError("could not draw a regex in the requested size range")


# ----------------------------------------------------------------------------------------------
# sources and arrivals
# ----------------------------------------------------------------------------------------------

def sample_sources(n_vertices: int, k: int, seed: int) -> np.ndarray:
    """k distinct vertex ids drawn uniformly, ascending, uint32."""
    rng = np.random.default_rng(seed)
    k = min(k, n_vertices)
    return np.sort(rng.choice(n_vertices, size=k, replace=False)).astype(np.uint32)


def poisson_arrivals(rate_qps: float, n: int, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_qps, size=n))


def serve_requests(n: int, n_vertices: int, names: Sequence[str], seed: int,
                   slice_width: int = 4096) -> List[tuple]:
    """The serving stream's requests: about 40% single-source RPQs ("rpq_single", regex, sources),
    40% RPQs over a slice of slice_width consecutive sources ("rpq_slice", regex, sources) and 20%
    CRPQs of 2-3 atoms anchored at a random source s ("crpq", atoms, n_vars, binding): the chain
    s -r1-> y -r2-> z, the fork s -r1-> y, s -r2-> y, or the triangle s -r1-> y, y -r2-> z,
    s -r3-> z.  RPQ regexes come from random_regex (1-11 label occurrences, depth <= 4); CRPQ
    atoms draw 1-3 occurrences from the rarer half of the labels, whose closures stay small, so
    a chain's second atom does not start from most of the graph."""
    rng = np.random.default_rng(seed)
    n_slices = max(1, n_vertices // slice_width)
    out = []
    for _ in range(n):
        u = rng.random()
        if u < 0.4:
            out.append(("rpq_single", random_regex(rng, names),
                        np.array([int(rng.integers(0, n_vertices))], dtype=np.uint32)))
        elif u < 0.8:
            lo = int(rng.integers(0, n_slices)) * slice_width
            out.append(("rpq_slice", random_regex(rng, names),
                        np.arange(lo, min(n_vertices, lo + slice_width), dtype=np.uint32)))
        else:
            s = int(rng.integers(0, n_vertices))
            shape = int(rng.integers(0, 3))
            rare = list(names[len(names) // 2:]) or list(names)
            r = [random_regex(rng, rare, max_leaves=3) for _ in range(3)]
            if shape == 0:
                out.append(("crpq", [(0, r[0], 1), (1, r[1], 2)], 3, [s, None, None]))
            elif shape == 1:
                out.append(("crpq", [(0, r[0], 1), (0, r[1], 1)], 2, [s, None]))
            else:
                out.append(("crpq", [(0, r[0], 1), (1, r[1], 2), (0, r[2], 2)], 3, [s, None, None]))
    return out


# ----------------------------------------------------------------------------------------------
# named workloads (sizes and seeds fixed here so every consumer draws the same bytes)
# ----------------------------------------------------------------------------------------------

WORKLOADS: Dict[str, dict] = {
    # all-pairs a.b.c* on a uniform random graph: 1,000 vertices, 5,000 edges, 4 labels
    "uniform_v1000_e5000_l4": dict(kind="uniform", n_vertices=1000, n_edges=5000, n_labels=4, seed=1,
                                   queries=["a.b.c*"]),
    # R-MAT scale 18 (262,144 vertices, 4,194,304 drawn edges), 8 labels Zipf(1.1)
    "rmat18_l8": dict(kind="rmat", scale=18, edge_factor=16, n_labels=8, zipf_s=1.1, seed=18,
                      queries=["a*", "a.b*", "(a|b).c*", "a.b*.c", "(a.b)*"]),
    # R-MAT scale 22 (4,194,304 vertices, 67,108,864 drawn edges), 16 labels Zipf(1.1)
    "rmat22_l16": dict(kind="rmat", scale=22, edge_factor=16, n_labels=16, zipf_s=1.1, seed=22),
    # typed social graph: 1M persons, 10M messages, 16,384 tags
    "social_p1m_m10m_t16k": dict(kind="social", seed=4),
    # R-MAT scale 23 (8,388,608 vertices, 134,217,728 drawn edges), 16 labels Zipf(1.1); the
    # throughput step runs the five Table 2 query shapes from a seeded sample of 65,536 sources
    # (all pairs at this scale take hours per step)
    "rmat23_l16": dict(kind="rmat", scale=23, edge_factor=16, n_labels=16, zipf_s=1.1, seed=23,
                       queries=["a*", "a.b*", "(a|b).c*", "a.b*.c", "(a.b)*"], bench_sources=65536),
}


def workload_graph(name: str, **overrides) -> EdgeList:
    """Draw the edge list of a named workload (keyword overrides allowed for
    scaled-down test variants)."""
    spec = dict(WORKLOADS[name])
    spec.update(overrides)
    kind = spec["kind"]
    if kind == "uniform":
        return uniform_graph(spec["n_vertices"], spec["n_edges"], spec["n_labels"], spec["seed"])
    if kind == "rmat":
        return rmat_graph(spec["scale"], spec.get("edge_factor", 16), n_labels=spec["n_labels"],
                          zipf_s=spec.get("zipf_s", 1.1), seed=spec["seed"])
    if kind == "social":
        keys = ("n_persons", "n_messages", "n_tags", "knows_mean_degree", "knows_gamma",
                "reply_p", "tag_zipf_s", "seed")
        return social_graph(**{k: spec[k] for k in keys if k in spec})
    raise KeyError(kind)


def rmat_query_mix(n_queries: int, n_vertices: int, names: Sequence[str], seed: int,
                   slice_width: int = 4096) -> List[Tuple[str, np.ndarray]]:
    """The batched mixed workload: query i even is single-source from a random
    vertex, query i odd is all-pairs over the source slice
    [slice_width*k, slice_width*(k+1)) for a seeded k.  Regexes have 1-11
    label occurrences and depth <= 4."""
    rng = np.random.default_rng(seed)
    out = []
    n_slices = max(1, n_vertices // slice_width)
    for i in range(n_queries):
        rx = random_regex(rng, names)
        if i % 2 == 0:
            src = np.array([int(rng.integers(0, n_vertices))], dtype=np.uint32)
        else:
            k = int(rng.integers(0, n_slices))
            lo = k * slice_width
            src = np.arange(lo, min(n_vertices, lo + slice_width), dtype=np.uint32)
        out.append((rx, src))
    return out
