"""Closed forms on the typed social graph (persons, messages, tags), computed from the edge
list with numpy/scipy alone: independent of the oracle and of the library.

* knows is symmetric, so knows.knows* (one or more knows steps) joins x and y exactly when they
  lie in one connected component of knows and each has a knows edge; a 3-cycle of such atoms over
  a person sample therefore holds the triples of sample persons inside one component, and their
  number is the sum over components of (sample persons with an edge in it) cubed.
* every message has one creator and one parent at most (replyOf), so the messages reached by
  replyOf* from m are m and its ancestors: depth(m) + 1 of them.
"""
import numpy as np


def knows_components(el, n_persons):
    """Connected components of the symmetric knows relation (scipy, independent of both sides)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    k = el.label == 0
    a = sp.coo_matrix((np.ones(int(k.sum()), dtype=np.int8), (el.src[k], el.dst[k])), shape=(n_persons, n_persons))
    _, comp = connected_components(a, directed=False)
    deg = np.bincount(el.src[k], minlength=n_persons)
    return comp, deg


def reply_depth(el, n_persons, n_messages):
    """Depth of every message in its reply tree (0 for roots), from the replyOf edges."""
    parent = np.full(n_messages, -1, dtype=np.int64)
    r = el.label == 2
    parent[el.src[r].astype(np.int64) - n_persons] = el.dst[r].astype(np.int64) - n_persons
    depth = np.zeros(n_messages, dtype=np.int64)
    cur = parent.copy()
    while True:
        live = cur >= 0
        if not live.any():
            break
        depth[live] += 1
        cur[live] = parent[cur[live]]
    return depth


def cycle_tuples(sample, comp, deg):
    """All (x, y, z) over the sample in one knows component, each with a knows edge: the
    tuples of the 3-cycle of knows.knows* atoms (knows is symmetric)."""
    s = np.sort(np.asarray(sample, dtype=np.int64))
    s = s[deg[s] > 0]
    out = []
    for c in np.unique(comp[s]):
        mem = s[comp[s] == c]
        x, y, z = np.meshgrid(mem, mem, mem, indexing="ij")
        out.append(np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1))
    if not out:
        return np.zeros((0, 3), dtype=np.int64)
    t = np.concatenate(out)
    return t[np.lexsort((t[:, 2], t[:, 1], t[:, 0]))]


def chain_hash(t):
    """Sum over rows of the chained mix m = mix64(v1), m = mix64(m ^ vi), modulo 2^64 (numpy)."""
    M = np.uint64

    def mix(x):
        z = (x + M(0x9E3779B97F4A7C15))
        z = (z ^ (z >> M(30))) * M(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> M(27))) * M(0x94D049BB133111EB)
        return z ^ (z >> M(31))
    with np.errstate(over="ignore"):
        t = t.astype(np.uint64)
        m = mix(t[:, 0])
        for j in range(1, t.shape[1]):
            m = mix(m ^ t[:, j])
        return int(m.sum(dtype=np.uint64))
