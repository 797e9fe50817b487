"""Reader for the small text fixtures under tests/golden/ (values printed in the paper)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_worked_example():
    names, vlabels, edges, pairs, query, n = None, None, [], [], None, None
    with open(os.path.join(GOLDEN, "worked_example.txt")) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "vertices":
                n = int(t[1])
            elif t[0] == "labels":
                names = t[1:]
            elif t[0] == "vertex_labels":
                vlabels = t[1:]
            elif t[0] == "edge":
                edges.append((int(t[1]), names.index(t[2]), int(t[3])))
            elif t[0] == "query":
                query = t[1]
            elif t[0] == "pair":
                pairs.append((int(t[1]), int(t[2])))
    e = np.array(edges, dtype=np.int64)
    vl_names = sorted(set(vlabels))
    vl = np.array([vl_names.index(x) for x in vlabels], dtype=np.uint8)
    return dict(n=n, names=names, src=e[:, 0].astype(np.uint32), label=e[:, 1].astype(np.uint8),
                dst=e[:, 2].astype(np.uint32), query=query, pairs=sorted(pairs),
                vertex_label=vl, vertex_label_names=vl_names)
