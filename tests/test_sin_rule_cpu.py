"""The solve kernel's label of s*_in, derived from the center labels, checked
on the CPU against the oracle's synchronous Bellman-Ford rounds.

s*_in (the anchor's copy that paths end at, Definitions of NCyc and NPath)
has no out-edges, so the kernel searches the centers only and derives its
label afterwards: best = min over u of dist[u] + w(u, s*_in); synchronous
rounds reach best one round after the earliest of its minimisers is fixed
(the smallest hop among them), and keep as predecessor the smallest
minimiser with that hop.  This test recomputes the center distances and hops
with plain synchronous rounds, applies that rule, and compares it with the
oracle's label and predecessor of s*_in, for NCyc (edges W[u][anchor]) and
NPath (penalty-difference edges, Appendix A)."""
import numpy as np
import pytest

import oracle
from tests import pins


def _table(rng, k):
    pot = rng.integers(-6, 7, size=k)
    W = np.full((k, k), pins.KEY_NONE, np.uint64)
    for u in range(k):
        for v in range(k):
            if u != v and rng.random() < 0.7:
                d = int(pot[v] - pot[u] + rng.integers(0, 3))
                W[u, v] = np.uint64(((d + 2**31) << 32) | int(rng.integers(0, 99)))
    return W


def center_labels(E, k, s):
    """Distances and hops (round in which each label is fixed) of synchronous
    rounds over the centers 0..k-1."""
    dist = {s: 0}
    hop = {s: 0}
    for t in range(1, k + 1):
        new = dict(dist)
        for (u, v), w in E.items():
            if v < k and u in dist and (v not in new or dist[u] + w < new[v]):
                new[v] = dist[u] + w               # candidates from the previous round
        changed = [v for v in new if v not in dist or new[v] < dist[v]]
        for v in changed:
            hop[v] = t
        dist = new
        if not changed:
            break
    return dist, hop


@pytest.mark.parametrize("seed", range(80))
def test_s_in_label_from_the_center_labels(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 10))
    W = _table(rng, k)
    s = int(rng.integers(0, k))
    mode = seed % 2
    load = rng.integers(0, 4, size=k).astype(np.int32)
    cap = rng.integers(0, 4, size=k).astype(np.int32)
    pen = rng.integers(1, 12, size=k).astype(np.int32)
    E = pins.split_graph(W, s, mode, load, cap, pen)
    dist, hop = center_labels(E, k, s)
    into = {u: w for (u, v), w in E.items() if v == k and u in dist}
    dist_o, pred_o, _ = oracle.refine_search(W, s, mode, load, cap, pen)
    if not into:
        assert dist_o[k] == oracle.DIST_NONE
        return
    best = min(dist[u] + w for u, w in into.items())
    mins = [u for u, w in into.items() if dist[u] + w == best]
    h = min(hop[u] for u in mins)
    pred = min(u for u in mins if hop[u] == h)
    assert (dist_o[k], pred_o[k]) == (best, pred), seed


@pytest.mark.parametrize("seed", range(40))
def test_path_search_reuses_the_cycle_search_labels(seed):
    """NCyc and NPath differ only in the edges into s*_in, so the center
    labels of the two searches are the same and the path search's answer is
    the rule above applied to the cycle search's labels."""
    rng = np.random.default_rng(1000 + seed)
    k = int(rng.integers(2, 10))
    W = _table(rng, k)
    s = int(rng.integers(0, k))
    load = rng.integers(0, 4, size=k).astype(np.int32)
    cap = rng.integers(0, 4, size=k).astype(np.int32)
    pen = rng.integers(1, 12, size=k).astype(np.int32)
    d0, p0, _ = oracle.refine_search(W, s, 0, load, cap, pen)
    d1, p1, _ = oracle.refine_search(W, s, 1, load, cap, pen)
    assert np.array_equal(d0[:k], d1[:k]) and np.array_equal(p0[:k], p1[:k])
    E = pins.split_graph(W, s, 1, load, cap, pen)
    dist, hop = center_labels(E, k, s)
    into = {u: w for (u, v), w in E.items() if v == k and u in dist}
    if not into:                                 # the anchor reaches no other center
        assert d1[k] == oracle.DIST_NONE
        return
    best = min(dist[u] + w for u, w in into.items())
    mins = [u for u, w in into.items() if dist[u] + w == best]
    h = min(hop[u] for u in mins)
    assert (d1[k], p1[k]) == (best, min(u for u in mins if hop[u] == h))
