"""The device's road-network searches (cost matrix from a road network,
Section 3.5 and the datasets of Section 5), modelled on the CPU.

Each center's search lowers vertex labels by atomic minima in rounds: a round
relaxes the arcs out of the vertices whose label dropped in the round before,
a relaxation reads its source's label at any moment after the previous
barrier, and a vertex whose label this relaxation lowered joins the next
frontier once (a round stamp taken by atomic exchange).  The claim is that,
whatever the interleaving, the labels end as the shortest distances, which
the oracle computes with Dijkstra's algorithm.  The model replays random
interleavings and stale reads on small graphs with zero-length arcs, parallel
arcs and unreachable vertices."""
import numpy as np
import pytest

import oracle

INF = 2**31 - 1


def _graph(rng, V):
    arcs = []
    for _ in range(int(rng.integers(V, 4 * V))):
        u, v = int(rng.integers(0, V)), int(rng.integers(0, V))
        arcs.append((u, v, int(rng.integers(0, 6))))   # zero lengths included
    arcs.sort()
    row_ptr = np.zeros(V + 1, np.int64)
    for u, _, _ in arcs:
        row_ptr[u + 1] += 1
    row_ptr = np.cumsum(row_ptr)
    col = np.array([a[1] for a in arcs], np.int32)
    length = np.array([a[2] for a in arcs], np.int32)
    return row_ptr, col, length


def rounds_model(row_ptr, col, length, src, rng):
    V = len(row_ptr) - 1
    dist = [INF] * V
    dist[src] = 0
    stamp = [None] * V
    stamp[src] = 0
    front = [src]
    for r in range(4 * V + 8):
        hist = [[x] for x in dist]             # values each label holds this round
        work = [(u, a) for u in front for a in range(row_ptr[u], row_ptr[u + 1])]
        rng.shuffle(work)
        nxt = []
        for u, a in work:
            du = hist[u][rng.integers(0, len(hist[u]))]   # any value since the barrier
            if du == INF:
                continue
            v = int(col[a])
            cand = du + int(length[a])
            old = dist[v]
            if cand < old:                      # this relaxation lowered the label
                dist[v] = cand
                hist[v].append(cand)
                if stamp[v] != r + 1:
                    stamp[v] = r + 1
                    nxt.append(v)
        if not nxt:
            return dist
        front = nxt
    raise AssertionError("round cap reached")


@pytest.mark.parametrize("seed", range(25))
def test_any_interleaving_gives_the_shortest_distances(seed):
    rng = np.random.default_rng(seed)
    V = int(rng.integers(2, 25))
    row_ptr, col, length = _graph(rng, V)
    src = int(rng.integers(0, V))
    # the oracle reports unreachable units as errors; ask only for the reached
    ref = np.full(V, INF, np.int64)
    seen, stack = {src}, [src]
    while stack:
        u = stack.pop()
        for a in range(row_ptr[u], row_ptr[u + 1]):
            if int(col[a]) not in seen:
                seen.add(int(col[a]))
                stack.append(int(col[a]))
    reach = sorted(seen)
    cm = oracle.road_cm(row_ptr, col, length, [src], reach)
    ref[reach] = cm[:, 0]
    for _ in range(6):
        assert rounds_model(row_ptr, col, length, src, rng) == [int(x) for x in ref]
