"""Pins of the oracle's CRPQ join (Definition 2) on a small typed social graph against closed
forms computed from the edge list alone (tests/social_forms.py): the 3-cycle of knows.knows*
atoms over a person sample, and the message/creator/reply-chain query."""
import numpy as np

import oracle
import synth
from social_forms import chain_hash, cycle_tuples, knows_components, reply_depth

P, M, T = 400, 1500, 64
PERSON, MESSAGE, TAG = 0, 1, 2


def small_social():
    return synth.social_graph(n_persons=P, n_messages=M, n_tags=T, knows_mean_degree=1.2, seed=11)


def test_three_cycle_is_sum_of_cubes():
    el = small_social()
    og = oracle.OracleGraph.from_edgelist(el)
    comp, deg = knows_components(el, P)
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(P, size=30, replace=False))
    cyc = [(0, "knows.knows*", 1), (1, "knows.knows*", 2), (2, "knows.knows*", 0)]
    got = oracle.crpq(og, cyc, 3, var_domain=[sample] * 3, var_label=[PERSON] * 3)
    want = cycle_tuples(sample, comp, deg)
    assert got == [tuple(int(v) for v in row) for row in want]
    live = sample[deg[sample] > 0]
    _, sizes = np.unique(comp[live], return_counts=True)
    assert len(got) == int((sizes ** 3).sum())
    assert oracle.crpq_hash(got) == chain_hash(want)
    # the sample has isolated persons and several components, so the form is not trivial
    assert (deg[sample] == 0).any() and len(sizes) > 1


def test_message_creator_reply_chain_count():
    el = small_social()
    og = oracle.OracleGraph.from_edgelist(el)
    tag1 = P + M
    atoms = [(0, "hasTag", 1), (0, "hasCreator", 2), (0, "replyOf*", 3)]
    got = oracle.crpq(og, atoms, 4, binding=[None, tag1, None, None], var_label=[MESSAGE, TAG, PERSON, MESSAGE])
    tagged = np.unique(el.src[(el.label == 3) & (el.dst == tag1)].astype(np.int64))
    depth = reply_depth(el, P, M)
    assert len(got) == int((depth[tagged - P] + 1).sum())
    assert sorted({t[0] for t in got}) == tagged.tolist()
    # creator column: the single hasCreator target of each message
    creator = {int(s): int(d) for s, l, d in zip(el.src, el.label, el.dst) if l == 1}
    assert all(creator[m] == u for (m, u, p) in got)
    assert depth[tagged - P].max() >= 2   # chains longer than one reply occur
