"""The solve kernel's search in Dijkstra order (used when node potentials
allow it), modelled on the CPU and checked against the oracle's synchronous
Bellman-Ford rounds.

With potentials pot feasible on every edge except those leaving the anchor s
(the search never enters s, so only its first hops may have negative reduced
weight w(u, v) + pot[u] - pot[v]), the kernel settles centers in the order of
(reduced label, edges) and keeps, per center, the smallest (distance, edges,
predecessor) offered by a settled center.  The claim: every center ends with
its shortest distance, the fewest edges among its shortest paths, and the
predecessor the synchronous rounds keep.  The model breaks ties between equal
keys at random."""
import numpy as np
import pytest

import oracle
from tests import pins


def _delta(key):
    return int(key >> np.uint64(32)) - 2**31


def _case(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 11))
    pot = rng.integers(-6, 7, size=k)
    W = np.full((k, k), pins.KEY_NONE, np.uint64)
    for u in range(k):
        for v in range(k):
            if u != v and rng.random() < 0.7:
                d = int(pot[v] - pot[u] + rng.integers(0, 3))
                W[u, v] = np.uint64(((d + 2**31) << 32) | int(rng.integers(0, 99)))
    s = int(rng.integers(0, k))
    for v in range(k):                          # the anchor's row may drop anywhere
        if v != s and W[s, v] != pins.KEY_NONE and rng.random() < 0.5:
            d = _delta(W[s, v]) - int(rng.integers(0, 8))
            W[s, v] = np.uint64(((d + 2**31) << 32) | int(rng.integers(0, 99)))
    return rng, k, pot, W, s


def dijkstra_order(W, s, pot, rng):
    k = W.shape[0]
    lab = {s: (0, 0, 0)}                        # (distance, edges, predecessor)
    settled = set()
    while True:
        open_ = [v for v in lab if v not in settled]
        if not open_:
            return lab
        # reduced label: the path's sum of w(u, v) + pot[u] - pot[v]
        key = {v: (lab[v][0] - pot[v] + pot[s], lab[v][1]) for v in open_}
        m = min(key.values())
        ties = [v for v in open_ if key[v] == m]
        u = ties[int(rng.integers(0, len(ties)))]
        settled.add(u)
        for v in range(k):
            if v == s or v in settled or W[u, v] == pins.KEY_NONE:
                continue
            cand = (lab[u][0] + _delta(W[u, v]), lab[u][1] + 1, u)
            if v not in lab or cand < lab[v]:
                lab[v] = cand


@pytest.mark.parametrize("seed", range(60))
def test_dijkstra_order_gives_the_synchronous_labels(seed):
    rng, k, pot, W, s = _case(seed)
    z = np.zeros(k, np.int32)
    dist, pred, _ = oracle.refine_search(W, s, 0, z, z, np.ones(k, np.int32))
    for _ in range(5):
        lab = dijkstra_order(W, s, pot, rng)
        for v in range(k):
            if v == s:
                continue
            if dist[v] == oracle.DIST_NONE:
                assert v not in lab
                continue
            assert (lab[v][0], lab[v][2]) == (dist[v], pred[v]), (seed, v)
