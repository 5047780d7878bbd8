"""The device search's frontier rounds, modelled on the CPU.

The solve kernel runs Bellman-Ford over the centers of the split graph
(Definitions of NCyc and NPath, Algorithm 1, Appendix A) with one barrier per
round: labels packed as (distance, edges, predecessor) are lowered by atomic
minima in whatever order the threads reach them, a relaxation reads its
source's label at some moment after the previous barrier, and a center whose
label drops enters the next round's frontier once (a round stamp).  The claim
that makes this exact is that the final labels do not depend on that order:
every center ends with its shortest distance and, as predecessor, the
smallest center that synchronous rounds would keep.

This model replays those rounds with random interleavings and random stale
reads and compares the labels with the oracle's synchronous rounds, on graphs
without a negative cycle (the invariant of Lemmas 1 and 2)."""
import numpy as np
import pytest

import oracle
from tests import pins

INF = (float("inf"), 0, 0)


def _graph(rng, k, spread):
    """A condensed table W with no negative cycle and many equal-cost ties:
    deltas are potential differences plus a small nonnegative slack."""
    pot = rng.integers(-spread, spread + 1, size=k)
    W = np.full((k, k), pins.KEY_NONE, np.uint64)
    for u in range(k):
        for v in range(k):
            if u == v or rng.random() < 0.25:
                continue
            d = int(pot[v] - pot[u] + rng.integers(0, 3))
            W[u, v] = np.uint64(((d + 2**31) << 32) | int(rng.integers(0, 1000)))
    return W


def _delta(key):
    return int(key >> np.uint64(32)) - 2**31


def frontier_rounds(W, s, rng):
    """Labels of the centers after the kernel's rounds, one interleaving."""
    k = W.shape[0]
    lab = [INF] * k
    lab[s] = (0, 0, 0)
    stamp = [0] * k
    front = [s]
    for t in range(1, k + 2):
        hist = [[x] for x in lab]              # values each label holds this round
        pairs = [(u, v) for u in front for v in range(k)
                 if v != s and W[u, v] != pins.KEY_NONE]
        rng.shuffle(pairs)
        nxt = []
        for u, v in pairs:
            lu = hist[u][rng.integers(0, len(hist[u]))]   # any value since the barrier
            if lu is INF:
                continue
            cand = (lu[0] + _delta(W[u, v]), lu[1] + 1, u)
            if cand < lab[v]:
                lab[v] = cand
                hist[v].append(cand)
                if stamp[v] != t:
                    stamp[v] = t
                    nxt.append(v)
        if not nxt:
            return lab, t
        front = nxt
    raise AssertionError("labels still dropping after k + 1 rounds")


@pytest.mark.parametrize("seed", range(30))
def test_any_interleaving_gives_the_synchronous_labels(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 13))
    W = _graph(rng, k, spread=int(rng.integers(0, 4)))
    s = int(rng.integers(0, k))
    z = np.zeros(k, np.int32)
    dist, pred, _ = oracle.refine_search(W, s, 0, z, z, np.ones(k, np.int32))
    for rep in range(8):
        lab, rounds = frontier_rounds(W, s, rng)
        assert rounds <= k + 1
        for v in range(k):
            if v == s:
                continue
            if dist[v] == oracle.DIST_NONE:
                assert lab[v] is INF
                continue
            d, e, p = lab[v]
            assert d == dist[v], (seed, rep, v)
            assert p == pred[v], (seed, rep, v)
            # edges: the length of the predecessor chain back to s
            n, x = 0, v
            while x != s:
                x = lab[x][2]
                n += 1
                assert n <= k
            assert e == n


def test_a_tie_keeps_the_smaller_predecessor_at_the_same_depth():
    """Two equal-cost paths of one edge each (via centers 1 and 2 into 3 after
    0 -> 1 and 0 -> 2): the label keeps center 1 whichever relaxation lands
    first, as the synchronous rounds do."""
    k = 4
    W = np.full((k, k), pins.KEY_NONE, np.uint64)

    def key(d):
        return np.uint64(((d + 2**31) << 32) | 7)

    W[0, 1] = key(2)
    W[0, 2] = key(2)
    W[2, 3] = key(1)
    W[1, 3] = key(1)
    rng = np.random.default_rng(1)
    z = np.zeros(k, np.int32)
    dist, pred, _ = oracle.refine_search(W, 0, 0, z, z, np.ones(k, np.int32))
    assert (dist[3], pred[3]) == (3, 1)
    for _ in range(20):
        lab, _ = frontier_rounds(W, 0, rng)
        assert lab[3] == (3, 2, 1)
