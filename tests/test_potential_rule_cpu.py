"""The solve kernel's node-potential checks, on the CPU against a check of
every edge.

Potentials certify that the best-transfer table has no negative cycle
(Lemmas 1 and 2 keep it so between refinements), which lets the kernel skip
searches exactly.  Two shortcuts decide whether a search's labels (distances
from the anchor s over the centers) are feasible potentials:
  * after a search that applied nothing, only the edges into s need checking:
    the Bellman-Ford fixpoint satisfies every edge between other centers;
  * after an applied refinement, only the rows of the centers it moved units
    between, and the edges into s, need checking: no other entry changed.
This test compares both shortcuts with the check of every edge."""
import numpy as np
import pytest

import oracle
from tests import pins


def _key(d):
    return np.uint64(((int(d) + 2**31) << 32) | 5)


def _table(rng, k, s):
    pot = rng.integers(-6, 7, size=k)
    W = np.full((k, k), pins.KEY_NONE, np.uint64)
    for u in range(k):
        for v in range(k):
            # the anchor holds a unit, so it has an edge to every center
            if u != v and (u == s or rng.random() < 0.7):
                W[u, v] = _key(pot[v] - pot[u] + rng.integers(0, 3))
    return W


def feasible(W, p, rows=None, col=None):
    """p[v] <= p[u] + W[u][v] on the edges of the given rows (all when None),
    or on the given column alone."""
    k = W.shape[0]
    for u in range(k):
        for v in range(k):
            if u == v or W[u, v] == pins.KEY_NONE:
                continue
            if col is not None and v != col:
                continue
            if col is None and rows is not None and u not in rows:
                continue
            if p[v] > p[u] + pins.key_delta(W[u, v]):
                return False
    return True


@pytest.mark.parametrize("seed", range(80))
def test_labels_need_only_the_checked_edges(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 10))
    s = int(rng.integers(0, k))
    W = _table(rng, k, s)
    if rng.random() < 0.5:                      # sometimes a negative cycle through s
        u = int(rng.integers(0, k))
        if u != s:
            W[u, s] = _key(pins.key_delta(W[s, u]) * -1 - int(rng.integers(1, 4)))
    z = np.zeros(k, np.int32)
    dist, _, _ = oracle.refine_search(W, s, 0, z, z, np.ones(k, np.int32))
    p = [int(dist[v]) for v in range(k)]
    # after a search that applied nothing: column s decides
    assert feasible(W, p) == feasible(W, p, col=s), seed
    # after an applied refinement: its centers' rows and column s decide
    moved = {int(c) for c in rng.choice(k, size=int(rng.integers(1, k + 1)), replace=False)}
    W2 = W.copy()
    for u in moved:
        for v in range(k):
            if u != v and rng.random() < 0.6:
                W2[u, v] = _key(int(rng.integers(-8, 9)))
            elif u != v and rng.random() < 0.2:
                W2[u, v] = pins.KEY_NONE
    full = feasible(W2, p)
    short = feasible(W2, p, rows=moved) and feasible(W2, p, col=s)
    assert full == short, seed


def _repair(W, p, tails):
    """The kernel's repair: labels start at 0 everywhere, the first round
    relaxes out of the tails of failed edges, later rounds out of the centers
    whose label dropped; returns p + lab shifted to p[s] + lab[s] = 0, or None
    without convergence."""
    k = W.shape[0]
    lab = [0] * k
    front = sorted(set(tails))
    for _ in range(k + 1):
        nxt = set()
        for u in front:
            for v in range(k):
                if u == v or W[u, v] == pins.KEY_NONE:
                    continue
                c = lab[u] + pins.key_delta(W[u, v]) + p[u] - p[v]
                if c < lab[v]:
                    lab[v] = c
                    nxt.add(v)
        if not nxt:
            return [p[v] + lab[v] for v in range(k)]
        front = sorted(nxt)
    return None


@pytest.mark.parametrize("seed", range(120))
def test_repair_from_failed_tails_restores_feasibility(seed):
    """After an applied refinement changes some rows, potentials that fail the
    check on those rows are repaired from the failed edges' tails alone; the
    result is feasible on every edge whenever the table has no negative cycle
    (Lemmas 1 and 2), and the repair then always converges."""
    rng = np.random.default_rng(1000 + seed)
    k = int(rng.integers(2, 10))
    s = int(rng.integers(0, k))
    W = _table(rng, k, s)
    z = np.zeros(k, np.int32)
    dist, _, _ = oracle.refine_search(W, s, 0, z, z, np.ones(k, np.int32))
    if any(dist[v] == oracle.DIST_NONE for v in range(k)) or not feasible(W, [int(x) for x in dist[:k]]):
        return                                   # a negative cycle through s: not this case
    p = [int(x) for x in dist[:k]]
    moved = {int(c) for c in rng.choice(k, size=int(rng.integers(1, k + 1)), replace=False)}
    W2 = W.copy()
    for u in moved:
        for v in range(k):
            if u != v and rng.random() < 0.6:
                W2[u, v] = _key(pins.key_delta(W[u, v]) - int(rng.integers(0, 6))
                                if W[u, v] != pins.KEY_NONE else int(rng.integers(-4, 9)))
    if pins.has_negative_cycle(W2):
        return
    rows = moved | {s}
    tails = [u for u in range(k) for v in range(k)
             if u != v and W2[u, v] != pins.KEY_NONE and (u in rows or v == s)
             and p[v] > p[u] + pins.key_delta(W2[u, v])]
    # the checked rows and column s hold every failed edge
    all_failed = [u for u in range(k) for v in range(k)
                  if u != v and W2[u, v] != pins.KEY_NONE and p[v] > p[u] + pins.key_delta(W2[u, v])]
    assert set(all_failed) <= set(tails)
    q = _repair(W2, p, tails)
    assert q is not None, seed
    assert feasible(W2, q), seed


def _sink_model(W, q):
    """The kernel's sink potentials: rounds from the sink over reversed edges,
    sigma(v) = min(q(v), min_w W[v][w] + sigma(w)), every center in the first
    frontier; None without convergence."""
    k = W.shape[0]
    sig = [int(x) for x in q]
    front = list(range(k))
    for _ in range(k + 1):
        nxt = set()
        for w in front:
            for v in range(k):
                if v == w or W[v, w] == pins.KEY_NONE:
                    continue
                c = sig[w] + pins.key_delta(W[v, w])
                if c < sig[v]:
                    sig[v] = c
                    nxt.add(v)
        if not nxt:
            return sig
        front = sorted(nxt)
    return None


@pytest.mark.parametrize("seed", range(80))
def test_sink_potentials_are_distances_to_the_sink_and_feasible(seed):
    """-sigma is a feasible potential, and sigma(v) is the cheapest cost of
    placing one more unit starting from v (brute force over simple paths);
    on such potentials the path search's bound term is smallest on the
    center that ends a cheapest path."""
    import itertools
    rng = np.random.default_rng(3000 + seed)
    k = int(rng.integers(2, 7))
    W = _table(rng, k, int(rng.integers(0, k)))
    if pins.has_negative_cycle(W):
        return
    q = rng.integers(0, 30, size=k)
    sig = _sink_model(W, q)
    assert sig is not None
    assert feasible(W, [-x for x in sig])
    for v in range(k):
        best = int(q[v])
        others = [u for u in range(k) if u != v]
        for r in range(1, k):
            for mid in itertools.permutations(others, r):
                path = (v,) + mid
                if any(W[a, b] == pins.KEY_NONE for a, b in zip(path, path[1:])):
                    continue
                cost = sum(pins.key_delta(W[a, b]) for a, b in zip(path, path[1:])) + int(q[path[-1]])
                best = min(best, cost)
        assert sig[v] == best, (seed, v)
