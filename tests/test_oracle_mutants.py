"""The oracle's pins must catch plausible mistakes in the oracle itself.

Each case below plants one mistake (a dropped term, a wrong index or sign, a
transposed operand, a missing reset, a wrong precedence) in a private copy of
``oracle/`` -- the C search, the automaton constructions or the CRPQ join --
and runs the pin suites (``test_oracle_pins.py``, ``test_oracle_crpq_forms.py``)
against that copy in a child process.  The case passes when at least one pin
fails on the planted mistake; an unmodified copy must pass every pin.

Everything here runs on the CPU and touches only temporary copies.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle_pins.py", "tests/test_oracle_crpq_forms.py"]
C = "rpq_oracle.c"
AUT = "automata.py"
INIT = "__init__.py"

# (name, [(file under oracle/, text to replace, replacement), ...])
MUTANTS = [
    # ---- the product-graph search (Definition 1, Section 2.2) -------------------------------
    ("zero-length walk not counted",
     [(C, "if (is_final[q] && !hit[s]) {", "if (0 && is_final[q] && !hit[s]) {")]),
    ("no epsilon closure after a move",
     [(C, "if (!eps_closure[(uint64_t)p * S + r]) continue;", "if (r != p) continue;")]),
    ("label range starts at the vertex's first edge",
     [(C, "uint64_t e = label_lower(g_lab, g_off[v], g_off[v + 1], l);", "uint64_t e = g_off[v];")]),
    ("edges of every label followed",
     [(C, "for (; e < g_off[v + 1] && g_lab[e] == l; ++e) {",
       "for (e = g_off[v]; e < g_off[v + 1]; ++e) {")]),
    ("edge followed backwards",
     [(C, "const uint32_t w = g_dst[e];", "const uint32_t w = v; (void)g_dst;")]),
    ("successor state ignored (stays in q)",
     [(C, "const uint32_t l = t_label[t], p = t_to[t];", "const uint32_t l = t_label[t], p = q; (void)t_to;")]),
    ("final state tested on the wrong state",
     [(C, "if (is_final[r] && !hit[w])", "if (is_final[p] && !hit[w])")]),
    ("visited set not cleared between sources",
     [(C, "for (uint64_t i = 0; i < queue.n; ++i) seen[queue.a[i]] = 0;", "")]),
    ("hit marks not cleared between sources",
     [(C, "for (uint64_t i = 0; i < found.n; ++i) hit[found.a[i]] = 0;", "")]),
    ("destinations left unsorted",
     [(C, "qsort(ys, (size_t)found.n, sizeof(uint32_t), cmp_u32);", "")]),
    ("pair key transposed",
     [(C, "const uint64_t key = ((uint64_t)s << 32) | ys[i];",
       "const uint64_t key = ((uint64_t)ys[i] << 32) | s;")]),
    ("checksum combined by xor",
     [(C, "h += oracle_splitmix64_output(key);", "h ^= oracle_splitmix64_output(key);")]),
    ("SplitMix64 shift constant",
     [(C, "z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;", "z = (z ^ (z >> 28)) * 0x94d049bb133111ebULL;")]),
    ("SplitMix64 increment dropped",
     [(C, "uint64_t z = state + 0x9e3779b97f4a7c15ULL;", "uint64_t z = state;")]),
    ("product edges counted per new (vertex, state)",
     [(C, "                    ++prod_edges;\n", ""),
      (C, "                        seen[idx] = 1;\n", "                        seen[idx] = 1; ++prod_edges;\n")]),
    ("product edges counted per transition, not per edge",
     [(C, "                    ++prod_edges;\n", ""),
      (C, "const uint32_t l = t_label[t], p = t_to[t];", "const uint32_t l = t_label[t], p = t_to[t]; ++prod_edges;")]),
    ("hop count off by one",
     [(C, "uint64_t head = 0, level_end = queue.n, hops = 0;",
       "uint64_t head = 0, level_end = queue.n, hops = 1;")]),
    ("length bound off by one",
     [(C, "if (hops >= max_len) continue;", "if (hops > max_len) continue;")]),
    ("length bound ignored",
     [(C, "if (hops >= max_len) continue;", "")]),
    ("duplicate edges kept",
     [(C, "if (i > b && key[i] == key[i - 1]) continue;", "")]),
    ("adjacency stores the source as the target",
     [(C, "key[pos[src[e]]++] = ((uint64_t)lab[e] << 32) | dst[e];",
       "key[pos[src[e]]++] = ((uint64_t)lab[e] << 32) | src[e];")]),
    ("labels sorted after targets in a vertex's list",
     [(C, "key[pos[src[e]]++] = ((uint64_t)lab[e] << 32) | dst[e];",
       "key[pos[src[e]]++] = ((uint64_t)dst[e] << 32) | lab[e];"),
      (C, "out_lab[out] = (uint32_t)(key[i] >> 32);", "out_lab[out] = (uint32_t)(key[i] & 0xffffffffULL);"),
      (C, "out_dst[out] = (uint32_t)(key[i] & 0xffffffffULL);", "out_dst[out] = (uint32_t)(key[i] >> 32);")]),
    # ---- parsing and the automata (Section 2.2) ------------------------------------------------
    ("postfix + read as *",
     [(AUT, '{"*": "star", "+": "plus", "?": "opt"}[k]', '{"*": "star", "+": "star", "?": "opt"}[k]')]),
    ("labels matched shortest-first",
     [(AUT, "order = sorted(range(len(names)), key=lambda i: -len(names[i]))",
       "order = sorted(range(len(names)), key=lambda i: len(names[i]))")]),
    ("union parsed tighter than concatenation",
     [(AUT, '            node = ("alt", node, p_cat())', '            node = ("alt", node, p_post())')]),
    ("Glushkov: star without its loop",
     [(AUT, "            for p in l:\n                follow[p] |= f\n            return (True if",
       "            return (True if")]),
    ("Glushkov: star not nullable",
     [(AUT, 'return (True if kind == "star" else n), f, l', "return n, f, l")]),
    ("Glushkov: first set of a concatenation tests the wrong operand",
     [(AUT, "(f1 | f2) if n1 else set(f1)", "(f1 | f2) if n2 else set(f1)")]),
    ("Glushkov: last set of a concatenation tests the wrong operand",
     [(AUT, "(l1 | l2) if n2 else set(l2)", "(l1 | l2) if n1 else set(l2)")]),
    ("Glushkov: concatenation nullable if either side is",
     [(AUT, "return (n1 and n2), ", "return (n1 or n2), ")]),
    ("Glushkov: follow of a concatenation reversed",
     [(AUT, "            for p in l1:\n                follow[p] |= f2",
       "            for p in l2:\n                follow[p] |= f1")]),
    ("Glushkov: initial state never final",
     [(AUT, "    if nullable:\n        finals.add(0)", "    pass")]),
    ("Thompson: option repeats",
     [(AUT, '            if kind in ("star", "plus"):\n                eps[f1].append(s1)',
       '            if kind in ("star", "plus", "opt"):\n                eps[f1].append(s1)')]),
    ("Thompson: plus may be skipped",
     [(AUT, '            if kind in ("star", "opt"):\n                eps[s].append(f)',
       '            if kind in ("star", "opt", "plus"):\n                eps[s].append(f)')]),
    ("Thompson: concatenation ends at its first part",
     [(AUT, "            eps[f1].append(s2)\n            return s1, f2",
       "            eps[f1].append(s2)\n            return s1, f1")]),
    ("epsilon closure takes one step only",
     [(AUT, "                        seen.add(y)\n                        stack.append(y)",
       "                        seen.add(y)")]),
    # ---- the CRPQ join (Definition 2) ------------------------------------------------------------
    ("vertex-label condition dropped",
     [(INIT, "d = d[g.vertex_label[d] == var_label[i]]", "d = d")]),
    ("distinctness filter dropped",
     [(INIT, "and assign[a] == assign[b]:\n                return False",
       "and assign[a] == assign[b]:\n                pass")]),
    ("join follows an atom in the wrong direction",
     [(INIT, "c = bwd[ai].get(assign[y], set())", "c = fwd[ai].get(assign[y], set())")]),
    ("atom targets filtered by the source variable's domain",
     [(INIT, "keep = np.isin(t, doms[y])", "keep = np.isin(t, doms[x])")]),
    ("atoms between assigned variables not re-checked",
     [(INIT, "            if ok_atoms(i) and ok_neq(i):", "            if ok_neq(i):")]),
    ("constants kept in the output tuple",
     [(INIT, "out.add(tuple(assign[j] for j in free))", "out.add(tuple(assign[j] for j in range(n_vars)))")]),
    ("constant binding ignored",
     [(INIT, "            d = np.array([binding[i]], dtype=np.int64)", "            pass")]),
]


def _plant(work: str, edits) -> None:
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(work, "oracle"),
                    ignore=shutil.ignore_patterns("_build", "__pycache__"))
    for (fname, old, new) in edits:
        path = os.path.join(work, "oracle", fname)
        text = open(path).read()
        n = text.count(old)
        if n != 1:
            raise AssertionError("planting %r: expected one occurrence in %s, found %d" % (old, fname, n))
        open(path, "w").write(text.replace(old, new))


def _run_pins(work: str):
    # The child starts in `work`, so `import oracle` finds the planted copy first;
    # the repository root follows for `synth` and the golden fixtures.
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([work, ROOT]), PYTHONDONTWRITEBYTECODE="1")
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-p", "no:randomly", "--tb=no",
           "-rf", "-m", "not gpu", "-c", os.devnull, "--rootdir", ROOT] + [os.path.join(ROOT, f) for f in PIN_FILES]
    try:
        p = subprocess.run(cmd, cwd=work, env=env, capture_output=True, text=True, timeout=900)
    except subprocess.TimeoutExpired:
        return -1, "timed out"
    return p.returncode, p.stdout + p.stderr


def _one(case):
    name, edits = case
    with tempfile.TemporaryDirectory(prefix="oracle_mutant_") as work:
        _plant(work, edits)
        rc, out = _run_pins(work)
        probe = subprocess.run([sys.executable, "-c", "import oracle; print(oracle.__file__)"], cwd=work,
                               env=dict(os.environ, PYTHONPATH=os.pathsep.join([work, ROOT])),
                               capture_output=True, text=True, timeout=300)
        return name, rc, out, probe.stdout.strip()


@pytest.fixture(scope="module")
def outcomes():
    cases = [("unmodified copy", [])] + MUTANTS
    workers = max(1, min(6, (os.cpu_count() or 2) - 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return {name: (rc, out, where) for (name, rc, out, where) in ex.map(_one, cases)}


def test_unmodified_copy_passes_every_pin(outcomes):
    rc, out, where = outcomes["unmodified copy"]
    assert where.startswith(tempfile.gettempdir()) and "oracle_mutant_" in where, where
    assert rc == 0, out[-3000:]


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(outcomes, name):
    rc, out, where = outcomes[name]
    assert "oracle_mutant_" in where, where
    assert rc == 1 and "FAILED" in out, "no pin caught %r:\n%s" % (name, out[-3000:])
