"""Regular-expression parsing and automaton construction for the oracle.

TEST INFRASTRUCTURE ONLY: nothing in the HIP library imports this module.

Query syntax (the paper writes alternation as infix '+', Section 2.2 and
Table 2; here it is '|', and postfix '+' means one-or-more):

    alt  := cat ('|' cat)*
    cat  := post (('.' | '·')? post)*
    post := atom ('*' | '+' | '?')*
    atom := LABEL | '(' alt ')'

Label tokens are matched longest-first against the graph's label names, so
"abc*" over names {a, b, c} reads a.b.c*, and "knows.knows*" works with
multi-letter names.

Two constructions are provided, each written from its textbook definition:

* ``thompson``: Thompson's construction (CACM 1968), one fragment per AST node
  glued with epsilon moves; one start and one accept state.
* ``glushkov``: the position automaton (Glushkov 1961; Berry and Sethi 1986):
  state 0 plus one state per label occurrence, with transitions from the
  nullable / first / last / follow sets.  It has no epsilon moves and is the
  canonical automaton on which product edges are counted.

Both return an :class:`EpsNFA` that the C search runs unchanged.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Sequence, Set, Tuple


class RegexSyntaxError(ValueError):
    pass


# AST nodes: ("lab", id) ("cat", a, b) ("alt", a, b) ("star", a) ("plus", a) ("opt", a)


def tokenize(text: str, names: Sequence[str]) -> List[Tuple[str, object]]:
    order = sorted(range(len(names)), key=lambda i: -len(names[i]))
    toks: List[Tuple[str, object]] = []
    i = 0
    while i < len(text):
        c = text[i]
        if c.isspace():
            i += 1
            continue
        if c in "|()*+?":
            toks.append((c, None))
            i += 1
            continue
        if c in ".·":
            toks.append((".", None))
            i += 1
            continue
        for li in order:
            nm = names[li]
            if nm and text.startswith(nm, i):
                toks.append(("L", li))
                i += len(nm)
                break
        else:
            raise RegexSyntaxError("unknown label at %r" % text[i:])
    return toks


def parse(text: str, names: Sequence[str]):
    toks = tokenize(text, names)
    pos = 0

    def peek():
        return toks[pos][0] if pos < len(toks) else None

    def eat(kind):
        nonlocal pos
        if peek() != kind:
            raise RegexSyntaxError("expected %r in %r" % (kind, text))
        pos += 1

    def p_alt():
        node = p_cat()
        while peek() == "|":
            eat("|")
            node = ("alt", node, p_cat())
        return node

    def p_cat():
        node = p_post()
        while True:
            k = peek()
            if k == ".":
                eat(".")
                node = ("cat", node, p_post())
            elif k in ("L", "("):
                node = ("cat", node, p_post())
            else:
                return node

    def p_post():
        node = p_atom()
        while peek() in ("*", "+", "?"):
            k = peek()
            eat(k)
            node = ({"*": "star", "+": "plus", "?": "opt"}[k], node)
        return node

    def p_atom():
        nonlocal pos
        k = peek()
        if k == "L":
            lid = toks[pos][1]
            pos += 1
            return ("lab", lid)
        if k == "(":
            eat("(")
            node = p_alt()
            eat(")")
            return node
        raise RegexSyntaxError("unexpected %r in %r" % (k, text))

    if not toks:
        raise RegexSyntaxError("empty query")
    tree = p_alt()
    if pos != len(toks):
        raise RegexSyntaxError("trailing input in %r" % text)
    return tree


@dataclasses.dataclass
class EpsNFA:
    """Automaton with labelled and epsilon moves.

    ``trans[q]`` is a list of (label, target); ``eps[q]`` a list of targets."""
    n_states: int
    start: int
    finals: Set[int]
    trans: List[List[Tuple[int, int]]]
    eps: List[List[int]]

    def closure(self) -> List[Set[int]]:
        out = []
        for q in range(self.n_states):
            seen = {q}
            stack = [q]
            while stack:
                x = stack.pop()
                for y in self.eps[x]:
                    if y not in seen:
                        seen.add(y)
                        stack.append(y)
            out.append(seen)
        return out

    def accepts(self, word: Sequence[int]) -> bool:
        """Direct simulation on a label word (used by the oracle's own tests)."""
        cl = self.closure()
        cur = set(cl[self.start])
        for a in word:
            nxt = set()
            for q in cur:
                for (l, p) in self.trans[q]:
                    if l == a:
                        nxt |= cl[p]
            cur = nxt
        return bool(cur & self.finals)


def thompson(tree) -> EpsNFA:
    trans: List[List[Tuple[int, int]]] = []
    eps: List[List[int]] = []

    def new():
        trans.append([])
        eps.append([])
        return len(trans) - 1

    def build(t):
        kind = t[0]
        if kind == "lab":
            s, f = new(), new()
            trans[s].append((t[1], f))
            return s, f
        if kind == "cat":
            s1, f1 = build(t[1])
            s2, f2 = build(t[2])
            eps[f1].append(s2)
            return s1, f2
        if kind == "alt":
            s, f = new(), new()
            s1, f1 = build(t[1])
            s2, f2 = build(t[2])
            eps[s] += [s1, s2]
            eps[f1].append(f)
            eps[f2].append(f)
            return s, f
        if kind in ("star", "plus", "opt"):
            s, f = new(), new()
            s1, f1 = build(t[1])
            eps[s].append(s1)
            eps[f1].append(f)
            if kind in ("star", "plus"):
                eps[f1].append(s1)          # repeat
            if kind in ("star", "opt"):
                eps[s].append(f)            # skip
            return s, f
        raise ValueError(kind)

    s, f = build(tree)
    return EpsNFA(len(trans), s, {f}, trans, eps)


def glushkov(tree) -> EpsNFA:
    """Position automaton: state 0 is initial, state p >= 1 is the p-th label
    occurrence from the left.  delta(0, l) = first positions labelled l,
    delta(p, l) = follow(p) positions labelled l; finals are the last
    positions, plus 0 when the expression accepts the empty word."""
    labels: List[int] = [-1]                 # labels[p] for p >= 1
    follow: Dict[int, Set[int]] = {}

    def walk(t):
        kind = t[0]
        if kind == "lab":
            labels.append(t[1])
            p = len(labels) - 1
            follow[p] = set()
            return False, {p}, {p}
        if kind == "cat":
            n1, f1, l1 = walk(t[1])
            n2, f2, l2 = walk(t[2])
            for p in l1:
                follow[p] |= f2
            return (n1 and n2), (f1 | f2) if n1 else set(f1), (l1 | l2) if n2 else set(l2)
        if kind == "alt":
            n1, f1, l1 = walk(t[1])
            n2, f2, l2 = walk(t[2])
            return (n1 or n2), f1 | f2, l1 | l2
        if kind in ("star", "plus"):
            n, f, l = walk(t[1])
            for p in l:
                follow[p] |= f
            return (True if kind == "star" else n), f, l
        if kind == "opt":
            n, f, l = walk(t[1])
            return True, f, l
        raise ValueError(kind)

    nullable, first, last = walk(tree)
    n = len(labels)
    trans: List[List[Tuple[int, int]]] = [[] for _ in range(n)]
    for p in sorted(first):
        trans[0].append((labels[p], p))
    for q in range(1, n):
        for p in sorted(follow[q]):
            trans[q].append((labels[p], p))
    finals = set(last)
    if nullable:
        finals.add(0)
    return EpsNFA(n, 0, finals, trans, [[] for _ in range(n)])


def leaf_count(tree) -> int:
    if tree[0] == "lab":
        return 1
    return sum(leaf_count(c) for c in tree[1:])


def reverse_tree(tree):
    """The expression for the reversed language."""
    kind = tree[0]
    if kind == "lab":
        return tree
    if kind == "cat":
        return ("cat", reverse_tree(tree[2]), reverse_tree(tree[1]))
    if kind == "alt":
        return ("alt", reverse_tree(tree[1]), reverse_tree(tree[2]))
    return (kind, reverse_tree(tree[1]))


def to_text(tree, names: Sequence[str]) -> str:
    """Fully parenthesised printing (for tests that build trees directly)."""
    kind = tree[0]
    if kind == "lab":
        return names[tree[1]]
    if kind == "cat":
        return "(%s.%s)" % (to_text(tree[1], names), to_text(tree[2], names))
    if kind == "alt":
        return "(%s|%s)" % (to_text(tree[1], names), to_text(tree[2], names))
    return "(%s)%s" % (to_text(tree[1], names), {"star": "*", "plus": "+", "opt": "?"}[kind])
