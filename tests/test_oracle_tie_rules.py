"""Pins of the oracle's predecessor tie rule (reading R6(d): Bellman-Ford in
synchronous rounds keeps the smallest node attaining a label) by brute force.

Enumerating every simple path from the anchor gives each node its shortest
distance d(v) and the fewest edges h(v) among its shortest paths.
Synchronous rounds fix v's label in round h(v), from the smallest u with
d(u) + w(u, v) = d(v) and h(u) = h(v) - 1; the oracle's search must report
exactly that predecessor, for the centers and for s*_in, on NCyc and NPath
(Sections 3.3-3.4, Appendix A) of tie-heavy tables."""
import itertools

import numpy as np
import pytest

import oracle
from tests import pins


def _table(rng, k):
    pot = rng.integers(-3, 4, size=k)
    W = np.full((k, k), pins.KEY_NONE, np.uint64)
    for u in range(k):
        for v in range(k):
            if u != v and rng.random() < 0.75:
                d = int(pot[v] - pot[u] + rng.integers(0, 2))     # many equal costs
                W[u, v] = np.uint64(((d + 2**31) << 32) | int(rng.integers(0, 50)))
    return W


def brute_labels(E, k, s):
    """d(v) and h(v) over all simple paths from s (nodes 0..k, k = s*_in,
    which has no out-edges)."""
    d, h = {s: 0}, {s: 0}
    others = [v for v in range(k + 1) if v != s]
    for L in range(1, len(others) + 1):
        for mid in itertools.permutations(others, L):
            if k in mid[:-1]:
                continue
            nodes = (s, *mid)
            cost, ok = 0, True
            for a, b in zip(nodes, nodes[1:]):
                if (a, b) not in E:
                    ok = False
                    break
                cost += E[(a, b)]
            if not ok:
                continue
            v, e = nodes[-1], len(nodes) - 1
            if v not in d or (cost, e) < (d[v], h[v]):
                d[v], h[v] = cost, e
    return d, h


@pytest.mark.parametrize("seed", range(60))
def test_predecessor_is_the_smallest_in_the_fixing_round(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 7))
    W = _table(rng, k)
    s = int(rng.integers(0, k))
    mode = seed % 2
    load = rng.integers(0, 3, size=k).astype(np.int32)
    cap = rng.integers(0, 3, size=k).astype(np.int32)
    pen = rng.integers(1, 6, size=k).astype(np.int32)
    E = pins.split_graph(W, s, mode, load, cap, pen)
    d, h = brute_labels(E, k, s)
    dist, pred, _ = oracle.refine_search(W, s, mode, load, cap, pen)
    for v in range(k + 1):
        if v == s:
            continue
        if v not in d:
            assert dist[v] == oracle.DIST_NONE
            continue
        want = min(u for (u, x), w in E.items()
                   if x == v and u in d and d[u] + w == d[v] and h[u] == h[v] - 1)
        assert (dist[v], pred[v]) == (d[v], want), (seed, v)
