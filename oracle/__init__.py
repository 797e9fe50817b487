"""CPU oracle for RPQ and CRPQ evaluation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2602_20748_amd``) and never imports it; both read their inputs from
``synth`` (seeded generators with no evaluation arithmetic).

* :func:`rpq` evaluates Definition 1 (paper, Section 2.1) by a per-source
  breadth-first search over the product of the graph and an automaton
  (Section 2.2, automata-based approach), in plain C (``rpq_oracle.c``).
  With ``automaton="thompson"`` it runs Thompson's epsilon-NFA; with
  ``"glushkov"`` (default) the position automaton, on which the number of
  product edges examined is the canonical work measure.
* :func:`crpq` evaluates Definition 2: every atom's pair set, then a plain
  backtracking join over the query variables in their declared order, with
  the vertex-label condition, constants, optional explicit domains and
  distinctness filters (Section 8.1 uses the latter in two queries).
* :func:`crpq_forward` evaluates the same definition for queries whose atoms
  all point from an earlier-declared variable to a later one, evaluating each
  atom only from the values its source variable takes (anchored queries on
  large graphs).
* :func:`mix64` is the per-key checksum (one SplitMix64 output).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import automata
from .automata import EpsNFA, glushkov, parse, thompson

__all__ = ["OracleGraph", "OracleResult", "rpq", "crpq", "crpq_forward", "crpq_bruteforce", "mix64",
           "compile_automaton", "build_library", "automata"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_LIB_DIR, "liboracle.so")
_lib = None
_lib_lock = threading.Lock()

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build_library(force: bool = True) -> str:
    """Compile rpq_oracle.c with gcc -O2 into oracle/_build/liboracle.so."""
    os.makedirs(_LIB_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp,
                               os.path.join(_HERE, "rpq_oracle.c")])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build_library(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            lib.oracle_mix64.restype = ctypes.c_uint64
            lib.oracle_mix64.argtypes = [ctypes.c_uint64]
            lib.oracle_hash_keys.restype = ctypes.c_uint64
            lib.oracle_hash_keys.argtypes = [_u64p, ctypes.c_uint64]
            lib.oracle_graph_build.restype = ctypes.c_uint64
            lib.oracle_graph_build.argtypes = [ctypes.c_uint32, ctypes.c_uint64, _u32p, _u8p, _u32p,
                                               _u64p, _u32p, _u32p]
            lib.oracle_rpq_eval.restype = ctypes.c_int
            lib.oracle_rpq_eval.argtypes = [ctypes.c_uint32, _u64p, _u32p, _u32p, ctypes.c_uint32,
                                            ctypes.c_uint32, _u8p, _u32p, _u32p, _u32p, _u8p, _u32p,
                                            ctypes.c_uint64, _u64p, ctypes.c_uint64, _u64p, _u64p,
                                            ctypes.c_uint64]
            _lib = lib
    return _lib


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def mix64(x: int) -> int:
    return int(_load().oracle_mix64(ctypes.c_uint64(int(x) & 0xFFFFFFFFFFFFFFFF)))


def hash_keys(keys) -> int:
    """Checksum of a key array: sum of mix64(key) modulo 2^64 (the result hash of a pair set)."""
    a = np.ascontiguousarray(keys).view(np.uint64)
    return int(_load().oracle_hash_keys(_ptr(a, _u64p), a.size))


class OracleGraph:
    """The oracle's own adjacency: distinct (label, dst) per vertex, sorted."""

    def __init__(self, n_vertices: int, src, label, dst, n_labels: Optional[int] = None,
                 names: Optional[Sequence[str]] = None, vertex_label=None):
        src = np.ascontiguousarray(src, dtype=np.uint32)
        label = np.ascontiguousarray(label, dtype=np.uint8)
        dst = np.ascontiguousarray(dst, dtype=np.uint32)
        if src.size and (int(src.max()) >= n_vertices or int(dst.max()) >= n_vertices):
            raise ValueError("vertex id out of range")
        E = src.shape[0]
        self.n_vertices = int(n_vertices)
        self.n_labels = int(n_labels if n_labels is not None else (int(label.max()) + 1 if E else 1))
        self.names = list(names) if names is not None else [chr(97 + i) for i in range(self.n_labels)]
        self.vertex_label = None if vertex_label is None else np.asarray(vertex_label, dtype=np.int64)
        self.off = np.zeros(n_vertices + 1, dtype=np.uint64)
        lab_out = np.zeros(max(E, 1), dtype=np.uint32)
        dst_out = np.zeros(max(E, 1), dtype=np.uint32)
        n = _load().oracle_graph_build(self.n_vertices, E, _ptr(src, _u32p), _ptr(label, _u8p),
                                       _ptr(dst, _u32p), _ptr(self.off, _u64p),
                                       _ptr(lab_out, _u32p), _ptr(dst_out, _u32p))
        self.n_edges = int(n)
        self.lab = np.ascontiguousarray(lab_out[:max(n, 1)])
        self.dst = np.ascontiguousarray(dst_out[:max(n, 1)])

    @classmethod
    def from_edgelist(cls, el) -> "OracleGraph":
        return cls(el.n_vertices, el.src, el.label, el.dst, el.n_labels, el.names,
                   getattr(el, "vertex_label", None))

    def edges(self) -> List[Tuple[int, int, int]]:
        out = []
        for v in range(self.n_vertices):
            for e in range(int(self.off[v]), int(self.off[v + 1])):
                out.append((v, int(self.lab[e]), int(self.dst[e])))
        return out


@dataclasses.dataclass
class OracleResult:
    pairs: Optional[np.ndarray]      # uint64 keys src<<32|dst, source-major ascending
    count: int
    hash: int
    per_source: np.ndarray           # uint64 [n_sources, 2] (count, hash)
    product_edges: int
    max_hops: int
    n_states: int


def compile_automaton(regex, names: Sequence[str], automaton: str = "glushkov") -> EpsNFA:
    tree = parse(regex, names) if isinstance(regex, str) else regex
    if automaton == "glushkov":
        return glushkov(tree)
    if automaton == "thompson":
        return thompson(tree)
    raise ValueError(automaton)


def _flatten(nfa: EpsNFA):
    S = nfa.n_states
    t_off = np.zeros(S + 1, dtype=np.uint32)
    t_lab, t_to = [], []
    for q in range(S):
        for (l, p) in nfa.trans[q]:
            t_lab.append(l)
            t_to.append(p)
        t_off[q + 1] = len(t_lab)
    cl = np.zeros((S, S), dtype=np.uint8)
    for q, c in enumerate(nfa.closure()):
        for r in c:
            cl[q, r] = 1
    fin = np.zeros(S, dtype=np.uint8)
    for f in nfa.finals:
        fin[f] = 1
    return (t_off, np.asarray(t_lab or [0], dtype=np.uint32), np.asarray(t_to or [0], dtype=np.uint32),
            np.ascontiguousarray(cl.reshape(-1)), fin)


_UNBOUNDED = 0xFFFFFFFFFFFFFFFF


def _run(g: OracleGraph, flat, start, S, sources: np.ndarray, want_pairs: bool, cap: int,
         max_len: int = _UNBOUNDED):
    t_off, t_lab, t_to, cl, fin = flat
    n = sources.shape[0]
    per = np.zeros((max(n, 1), 2), dtype=np.uint64)
    totals = np.zeros(4, dtype=np.uint64)
    pairs = np.zeros(max(cap, 1), dtype=np.uint64) if want_pairs else None
    rc = _load().oracle_rpq_eval(
        g.n_vertices, _ptr(g.off, _u64p), _ptr(g.lab, _u32p), _ptr(g.dst, _u32p), S, start,
        _ptr(fin, _u8p), _ptr(t_off, _u32p), _ptr(t_lab, _u32p), _ptr(t_to, _u32p), _ptr(cl, _u8p),
        _ptr(sources, _u32p), n, _ptr(pairs, _u64p) if want_pairs else None, cap if want_pairs else 0,
        _ptr(per, _u64p), _ptr(totals, _u64p), max_len)
    if rc != 0:
        raise MemoryError("oracle ran out of memory")
    return pairs, per[:n], totals


def rpq(g: OracleGraph, regex, sources=None, automaton: str = "glushkov", pairs: bool = True,
        threads: int = 1, max_pairs: int = 1 << 26, max_length: Optional[int] = None) -> OracleResult:
    """Evaluate one RPQ from the given sources (default: every vertex).

    Sources must be distinct; results are emitted in the given source order
    (ascending keys when sources are ascending).  max_length = k keeps only
    walks of at most k edges (a length-bounded RPQ, the extension named in the
    paper's conclusion); None means walks of any length (Definition 1)."""
    ml = _UNBOUNDED if max_length is None else int(max_length)
    if ml < 0:
        raise ValueError("max_length must be >= 0")
    nfa = regex if isinstance(regex, EpsNFA) else compile_automaton(regex, g.names, automaton)
    flat = _flatten(nfa)
    if sources is None:
        sources = np.arange(g.n_vertices, dtype=np.uint32)
    sources = np.ascontiguousarray(sources, dtype=np.uint32)
    if sources.size and int(sources.max()) >= g.n_vertices:
        raise ValueError("source out of range")
    n = sources.shape[0]
    threads = max(1, min(int(threads), max(n, 1)))
    chunks = np.array_split(sources, threads) if threads > 1 else [sources]

    def job(chunk):
        if not pairs:
            return _run(g, flat, nfa.start, nfa.n_states, chunk, False, 0, ml)
        # first pass sizes the pair buffer exactly
        _, per, _t = _run(g, flat, nfa.start, nfa.n_states, chunk, False, 0, ml)
        need = int(per[:, 0].sum()) if chunk.size else 0
        if need > max_pairs:
            raise MemoryError("oracle result larger than max_pairs")
        return _run(g, flat, nfa.start, nfa.n_states, chunk, True, need, ml)

    if threads == 1:
        outs = [job(chunks[0])]
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            outs = list(ex.map(job, chunks))
    per = np.concatenate([o[1] for o in outs]) if n else np.zeros((0, 2), np.uint64)
    totals = [o[2] for o in outs]
    count = int(sum(int(t[0]) for t in totals))
    h = int(sum(int(t[1]) for t in totals)) & 0xFFFFFFFFFFFFFFFF
    pe = int(sum(int(t[2]) for t in totals))
    mh = int(max(int(t[3]) for t in totals)) if totals else 0
    pr = None
    if pairs:
        parts = [o[0][: int(o[1][:, 0].sum())] for o in outs if o[0] is not None]
        pr = np.concatenate(parts) if parts else np.zeros(0, np.uint64)
    return OracleResult(pr, count, h, per, pe, mh, nfa.n_states)


def pair_set(res: OracleResult) -> set:
    return {(int(k) >> 32, int(k) & 0xFFFFFFFF) for k in res.pairs}


# ------------------------------------------------------------------------------------------------
# CRPQ (Definition 2): atoms, then a plain join over the variables in declared order
# ------------------------------------------------------------------------------------------------

def _domains(g: OracleGraph, n_vars, binding, var_label, var_domain):
    doms: List[Optional[np.ndarray]] = []
    for i in range(n_vars):
        d = np.arange(g.n_vertices, dtype=np.int64)
        if binding is not None and binding[i] is not None and binding[i] >= 0:
            d = np.array([binding[i]], dtype=np.int64)
        if var_label is not None and var_label[i] is not None and var_label[i] >= 0:
            if g.vertex_label is None:
                raise ValueError("graph has no vertex labels")
            d = d[g.vertex_label[d] == var_label[i]]
        if var_domain is not None and var_domain[i] is not None:
            d = np.intersect1d(d, np.asarray(var_domain[i], dtype=np.int64))
        doms.append(d)
    return doms


def crpq_atom_relations(g: OracleGraph, atoms, doms, threads=1):
    rels = []
    for (x, rx, y) in atoms:
        res = rpq(g, rx, sources=doms[x].astype(np.uint32), threads=threads)
        k = res.pairs.astype(np.uint64)
        s = (k >> np.uint64(32)).astype(np.int64)
        t = (k & np.uint64(0xFFFFFFFF)).astype(np.int64)
        keep = np.isin(t, doms[y])
        rels.append((s[keep], t[keep]))
    return rels


def crpq(g: OracleGraph, atoms: Sequence[Tuple[int, str, int]], n_vars: int, binding=None,
         var_label=None, neq: Sequence[Tuple[int, int]] = (), var_domain=None,
         threads: int = 1) -> List[Tuple[int, ...]]:
    """Distinct tuples of the free variables (those without a constant), in
    declared order, sorted lexicographically."""
    doms = _domains(g, n_vars, binding, var_label, var_domain)
    rels = crpq_atom_relations(g, atoms, doms, threads)
    fwd: List[Dict[int, set]] = []
    bwd: List[Dict[int, set]] = []
    for (s, t) in rels:
        f: Dict[int, set] = {}
        b: Dict[int, set] = {}
        for a, c in zip(s.tolist(), t.tolist()):
            f.setdefault(a, set()).add(c)
            b.setdefault(c, set()).add(a)
        fwd.append(f)
        bwd.append(b)
    free = [i for i in range(n_vars) if not (binding is not None and binding[i] is not None and binding[i] >= 0)]
    out = set()
    assign: List[Optional[int]] = [None] * n_vars
    dom_sets = [set(d.tolist()) for d in doms]   # built once; candidates() intersects with them

    def candidates(i):
        cand = None
        for ai, (x, _, y) in enumerate(atoms):
            if x == i and y == i:
                continue
            if x == i and assign[y] is not None:
                c = bwd[ai].get(assign[y], set())
            elif y == i and assign[x] is not None:
                c = fwd[ai].get(assign[x], set())
            else:
                continue
            cand = set(c) if cand is None else (cand & c)
        if cand is None:
            cand = dom_sets[i]
        else:
            cand = cand & dom_sets[i]
        return sorted(cand)

    def ok_atoms(i):
        for ai, (x, _, y) in enumerate(atoms):
            if assign[x] is None or assign[y] is None:
                continue
            if i not in (x, y):
                continue
            if assign[y] not in fwd[ai].get(assign[x], ()):
                return False
        return True

    def ok_neq(i):
        for (a, b) in neq:
            if i in (a, b) and assign[a] is not None and assign[b] is not None and assign[a] == assign[b]:
                return False
        return True

    def rec(i):
        if i == n_vars:
            out.add(tuple(assign[j] for j in free))
            return
        for v in candidates(i):
            assign[i] = v
            if ok_atoms(i) and ok_neq(i):
                rec(i + 1)
            assign[i] = None

    rec(0)
    return sorted(out)


def crpq_bruteforce(g: OracleGraph, atoms, n_vars, binding=None, var_label=None, neq=(),
                    var_domain=None) -> List[Tuple[int, ...]]:
    """Every assignment of every variable to every vertex, checked against
    Definition 2 directly (tiny graphs only)."""
    import itertools
    doms = _domains(g, n_vars, binding, var_label, var_domain)
    rel = []
    for (x, rx, y) in atoms:
        res = rpq(g, rx)
        rel.append(pair_set(res))
    free = [i for i in range(n_vars) if not (binding is not None and binding[i] is not None and binding[i] >= 0)]
    out = set()
    domsets = [set(d.tolist()) for d in doms]
    for f in itertools.product(range(g.n_vertices), repeat=n_vars):
        if any(f[i] not in domsets[i] for i in range(n_vars)):
            continue
        if any(f[a] == f[b] for (a, b) in neq):
            continue
        if all((f[x], f[y]) in rel[k] for k, (x, _, y) in enumerate(atoms)):
            out.add(tuple(f[j] for j in free))
    return sorted(out)


def crpq_hash(tuples: Sequence[Tuple[int, ...]]) -> int:
    """Checksum of a tuple set: sum over tuples of the chained mix
    m = mix64(x1); m = mix64(m ^ x_i) for later columns, modulo 2^64."""
    h = 0
    for t in tuples:
        m = mix64(t[0])
        for x in t[1:]:
            m = mix64(m ^ int(x))
        h = (h + m) & 0xFFFFFFFFFFFFFFFF
    return h


def crpq_forward(g: OracleGraph, atoms: Sequence[Tuple[int, str, int]], n_vars: int, binding=None,
                 var_label=None, neq: Sequence[Tuple[int, int]] = (), var_domain=None, threads: int = 1,
                 max_pairs: int = 1 << 28, max_rows: int = 1 << 24) -> List[Tuple[int, ...]]:
    """Definition 2 for queries in which every atom x -rho-> y has x declared no later than y
    (chains, forks and triangles anchored at a constant, for instance).

    The variables are bound one at a time in declared order, keeping every partial assignment
    that satisfies the conditions on the bound variables.  An atom's pair set is needed only
    from the values its source variable takes in those assignments, so it is evaluated (with
    :func:`rpq`) from exactly those sources; the result is the same tuple set as :func:`crpq`,
    without evaluating atoms from every vertex of a free variable's domain."""
    for (x, _, y) in atoms:
        if x > y:
            raise ValueError("crpq_forward needs every atom's source variable declared first")
    doms = _domains(g, n_vars, binding, var_label, var_domain)
    succ: List[Dict[int, np.ndarray]] = [dict() for _ in atoms]

    def targets_from(ai, values):
        # R(rho_ai) from every value not evaluated yet, split per source
        need = sorted(set(values) - succ[ai].keys())
        if not need:
            return
        res = rpq(g, atoms[ai][1], sources=np.array(need, dtype=np.uint32), threads=threads,
                  max_pairs=max_pairs)
        k = res.pairs.astype(np.uint64)
        s = (k >> np.uint64(32)).astype(np.int64)
        t = (k & np.uint64(0xFFFFFFFF)).astype(np.int64)
        bounds = np.searchsorted(s, np.array(need, dtype=np.int64), side="left")
        ends = np.searchsorted(s, np.array(need, dtype=np.int64), side="right")
        for v, b, e in zip(need, bounds, ends):
            succ[ai][v] = t[b:e]

    rows: List[Tuple[int, ...]] = [()]
    for i in range(n_vars):
        into = [ai for ai, (x, _, y) in enumerate(atoms) if y == i and x < i]
        loops = [ai for ai, (x, _, y) in enumerate(atoms) if x == i and y == i]
        for ai in into:
            targets_from(ai, {r[atoms[ai][0]] for r in rows})
        dom_i = doms[i]
        cand_rows = []
        for r in rows:
            cand = None
            for ai in into:
                c = succ[ai][r[atoms[ai][0]]]
                cand = c if cand is None else np.intersect1d(cand, c)
            cand = dom_i if cand is None else np.intersect1d(cand, dom_i)
            cand_rows.append(cand)
        if loops:
            vals = set()
            for c in cand_rows:
                vals.update(int(v) for v in c)
            for ai in loops:
                targets_from(ai, vals)
        new_rows: List[Tuple[int, ...]] = []
        for r, cand in zip(rows, cand_rows):
            for v in cand.tolist():
                if any(not np.isin(v, succ[ai][v]).item() for ai in loops):
                    continue
                if any((a == i and b < i and r[b] == v) or (b == i and a < i and r[a] == v) for (a, b) in neq):
                    continue
                new_rows.append(r + (v,))
        if len(new_rows) > max_rows:
            raise MemoryError("crpq_forward: more than max_rows partial assignments")
        rows = new_rows
    free = [i for i in range(n_vars) if not (binding is not None and binding[i] is not None and binding[i] >= 0)]
    return sorted({tuple(r[j] for j in free) for r in rows})
