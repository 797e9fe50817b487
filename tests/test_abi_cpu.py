"""CPU-side checks of the C ABI: the library loads, exports every declared
symbol, and its host-side query compiler agrees with the oracle's own
Glushkov construction (same language, same state count, same transitions).
No GPU compute is called here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2602_20748_amd as rpq
from oracle.automata import glushkov, parse, thompson
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "rpq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:rpq|crpq)_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    path = rpq.library_path()
    if not os.path.exists(path):
        from paper_2602_20748_amd import build
        build.build()
    return rpq.load_library()


def test_library_exports_every_declared_symbol(lib):
    declared = header_functions()
    assert declared, "no declarations parsed"
    assert sorted(rpq.EXPORTED_SYMBOLS) == declared
    for name in declared:
        assert hasattr(lib, name), name
    assert rpq.rpq_abi_version() == 2


def test_struct_sizes_match_header():
    assert ctypes.sizeof(rpq.Nfa) == 16 + 4 * 32 * 64
    assert ctypes.sizeof(rpq.EvalOpts) == 24


# ctypes mirror -> C struct of include/rpq.h
STRUCTS = [("Nfa", "rpq_nfa"), ("GraphInfo", "rpq_graph_info"), ("EvalOpts", "rpq_eval_opts"),
           ("_Result", "rpq_result"), ("Profile", "rpq_profile"), ("BatchOpts", "rpq_batch_opts"),
           ("BatchInfo", "rpq_batch_info"), ("CrpqAtom", "crpq_atom"), ("CrpqVars", "crpq_vars"),
           ("CrpqResult", "crpq_result"), ("ServerOpts", "rpq_server_opts"), ("Request", "rpq_request"),
           ("Ticket", "rpq_ticket"), ("ServerStats", "rpq_server_stats")]


def test_ctypes_layouts_match_the_c_header(tmp_path):
    """Compile a probe against include/rpq.h with the host C compiler and compare every
    struct size and field offset with the Python binding's ctypes mirrors."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc") or shutil.which("cc")
    if gcc is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rpq.h"', "int main(void) {"]
    for py, c in STRUCTS:
        cls = getattr(rpq, py)
        lines.append('  printf("%s %%zu\\n", sizeof(%s));' % (c, c))
        for f in cls._fields_:
            lines.append('  printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (c, f[0], c, f[0]))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run([gcc, "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                        "-I", "/opt/rocm/include", str(src), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    for py, c in STRUCTS:
        cls = getattr(rpq, py)
        assert int(got[c]) == ctypes.sizeof(cls), c
        for f in cls._fields_:
            assert int(got["%s.%s" % (c, f[0])]) == getattr(cls, f[0]).offset, (c, f[0])


def nfa_as_oracle_shape(nfa):
    trans = {}
    for q in range(nfa.n_states):
        for l in range(nfa.n_labels):
            m = nfa.successors(q, l)
            for p in range(32):
                if m >> p & 1:
                    trans.setdefault(q, set()).add((l, p))
    finals = {q for q in range(32) if nfa.final_mask >> q & 1}
    return nfa.n_states, trans, finals


def test_compiler_matches_oracle_glushkov(lib):
    names = ["a", "b", "c", "d"]
    rng = np.random.default_rng(123)
    queries = ["a.b.c*", "a*", "a.b*", "(a|b).c*", "a.b*.c", "(a.b)*", "a?b*", "abcd", "abc*", "(a|b)*"]
    for _ in range(200):
        queries.append(synth.random_regex(rng, names))
    for q in queries:
        nfa = rpq.rpq_nfa_compile(q, names)
        g = glushkov(parse(q, names))
        n, trans, finals = nfa_as_oracle_shape(nfa)
        assert n == g.n_states, q
        want = {qq: set(ts) for qq, ts in enumerate(g.trans) if ts}
        assert trans == want, q
        assert finals == g.finals, q
        assert nfa.initial_mask == 1


def test_compiler_state_count_abc_star(lib):
    assert rpq.rpq_nfa_compile("a.b.c*", ["a", "b", "c", "d"]).n_states == 4


def test_compiler_multichar_names_and_middle_dot(lib):
    names = ["knows", "hasCreator", "replyOf", "hasTag"]
    n1 = rpq.rpq_nfa_compile("knows.knows*", names)
    n2 = rpq.rpq_nfa_compile("knows·knows*", names)
    n3 = rpq.rpq_nfa_compile("knows knows*", names)
    for n in (n2, n3):
        assert bytes(n) == bytes(n1)
    assert n1.n_states == 3


@pytest.mark.parametrize("bad,code", [("", rpq.RPQ_EINVAL), ("a.(b", rpq.RPQ_EINVAL), ("x", rpq.RPQ_EINVAL),
                                      ("a|", rpq.RPQ_EINVAL), ("a" * 32, rpq.RPQ_EUNSUPPORTED)])
def test_compiler_errors(lib, bad, code):
    with pytest.raises(rpq.RpqError) as ei:
        rpq.rpq_nfa_compile(bad, ["a", "b"])
    assert ei.value.code == code
    assert rpq.rpq_last_error()


def test_reverse_automaton(lib):
    names = ["a", "b", "c"]
    nfa = rpq.rpq_nfa_compile("a.b*.c", names)
    r = rpq.rpq_nfa_reverse(nfa)
    assert r.initial_mask == nfa.final_mask and r.final_mask == nfa.initial_mask
    for q in range(nfa.n_states):
        for l in range(3):
            for p in range(nfa.n_states):
                assert bool(nfa.successors(q, l) >> p & 1) == bool(r.successors(p, l) >> q & 1)
    assert bytes(rpq.rpq_nfa_reverse(r)) == bytes(nfa)


def test_workspace_size_rejects_null_graph(lib):
    nfa = rpq.rpq_nfa_compile("a*", ["a"])
    n = ctypes.c_uint64()
    rc = lib.rpq_eval_workspace_size(None, ctypes.byref(nfa), 10, 0, None, ctypes.byref(n))
    assert rc == rpq.RPQ_EINVAL


def _table_accepts(nfa, word):
    cur = nfa.initial_mask
    for a in word:
        nxt = 0
        for q in range(nfa.n_states):
            if (cur >> q) & 1:
                nxt |= nfa.successors(q, a)
        cur = nxt
    return bool(cur & nfa.final_mask)


@pytest.mark.parametrize("regex", ["a", "a.b*", "(a|b).c*", "a?", "(a.b)*", "c*.a+"])
def test_append_label_accepts_the_language_then_the_label(lib, regex):
    # L(append(rho, lambda)) = L(rho) . lambda for a label lambda outside rho's alphabet: checked
    # word by word against the oracle's Thompson automaton for rho, over every word of length <= 5
    names = ["a", "b", "c"]
    nfa = rpq.rpq_nfa_compile(regex, names)
    ap = rpq.rpq_nfa_append_label(nfa, 3)
    assert ap.n_states == nfa.n_states + 1 and ap.n_labels == 4
    ref = thompson(parse(regex, names))
    words = [[]]
    for _ in range(5):
        words += [w + [a] for w in words if len(w) == _ for a in range(4)]
    for w in words:
        want = len(w) >= 1 and w[-1] == 3 and 3 not in w[:-1] and ref.accepts(w[:-1])
        assert _table_accepts(ap, w) == want, (regex, w)
    with pytest.raises(rpq.RpqError):
        rpq.rpq_nfa_append_label(nfa, 64)
