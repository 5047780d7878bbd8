"""Pins of the oracle's road-network cost matrix (construction of CM, Section
3.5; the paper's datasets, Section 5), independent of its code.

Shortest-path lengths have one right answer, so the oracle is pinned to
scipy's Dijkstra (a library routine) and to Floyd-Warshall written out here
on small graphs; at the full 65,902-vertex size its distances from every
center to every vertex satisfy the shortest-path certificate: the center is
at 0, no arc can shorten a label, and every other label is met by some
in-arc with equality (with non-negative lengths these labels are exactly the
shortest distances).
"""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import dijkstra

import lbdd_inputs as L
import oracle


def _random_graph(rng, V, p, two_way=True, lmax=50):
    arcs = {}
    for u in range(V):
        for v in range(V):
            if u != v and rng.random() < p:
                w = int(rng.integers(0, lmax))
                arcs[(u, v)] = w
                if two_way:
                    arcs[(v, u)] = w
    for u in range(V - 1):                       # a path keeps everything reachable
        arcs.setdefault((u, u + 1), int(rng.integers(0, lmax)))
        arcs.setdefault((u + 1, u), int(rng.integers(0, lmax)))
    keys = sorted(arcs)
    row_ptr = np.zeros(V + 1, np.int64)
    for u, _ in keys:
        row_ptr[u + 1] += 1
    row_ptr = np.cumsum(row_ptr)
    col = np.array([v for _, v in keys], np.int32)
    ln = np.array([arcs[x] for x in keys], np.int32)
    return row_ptr, col, ln


def _floyd(V, row_ptr, col, ln):
    D = np.full((V, V), np.iinfo(np.int64).max // 4, np.int64)
    np.fill_diagonal(D, 0)
    for u in range(V):
        for i in range(row_ptr[u], row_ptr[u + 1]):
            D[u, col[i]] = min(D[u, col[i]], ln[i])
    for m in range(V):
        D = np.minimum(D, D[:, m:m + 1] + D[m:m + 1, :])
    return D


@pytest.mark.parametrize("seed", range(20))
def test_small_graphs_equal_floyd_warshall(seed):
    rng = np.random.default_rng(seed)
    V = int(rng.integers(2, 14))
    rp, col, ln = _random_graph(rng, V, 0.25, two_way=bool(seed % 2))
    k = int(rng.integers(1, V + 1))
    centers = rng.choice(V, size=k, replace=False).astype(np.int32)
    units = rng.integers(0, V, size=int(rng.integers(1, 20))).astype(np.int32)
    cm = oracle.road_cm(rp, col, ln, centers, units)
    D = _floyd(V, rp, col, ln)
    assert np.array_equal(cm, D[np.ix_(centers, units)].T)


@pytest.mark.parametrize("seed", range(6))
def test_generated_networks_equal_scipy_dijkstra(seed):
    net = L.road_network(3000 + 37 * seed, 50 + seed, 12, seed=seed)
    cm = oracle.road_cm(net.row_ptr, net.col, net.length, net.centers, net.units)
    G = csr_matrix((net.length.astype(np.float64), net.col, net.row_ptr), shape=(net.V, net.V))
    D = dijkstra(G, indices=net.centers)
    assert np.array_equal(cm, D[:, net.units].T.astype(np.int64))


def certificate_ok(net, dist_all):
    """dist_all [V][k]: shortest-path lengths from every center, checked by the
    shortest-path certificate (see the module docstring)."""
    V = net.V
    src = np.repeat(np.arange(V), np.diff(net.row_ptr))
    dst = net.col.astype(np.int64)
    w = net.length.astype(np.int64)[:, None]
    D = dist_all.astype(np.int64)
    if not (D[net.centers, np.arange(net.k)] == 0).all():
        return False
    cand = D[src] + w                                  # [E][k]
    if (cand < D[dst]).any():
        return False                                   # some arc shortens a label
    best_in = np.full_like(D, np.iinfo(np.int64).max)
    np.minimum.at(best_in, dst, cand)
    met = best_in == D
    met[net.centers, np.arange(net.k)] = True
    return bool(met.all())


def test_r1_network_certificate():
    """The 65,902-vertex, 131-center network: distances to every vertex."""
    net = L.make_road_config("R1")
    all_v = np.arange(net.V, dtype=np.int32)
    D = oracle.road_cm(net.row_ptr, net.col, net.length, net.centers, all_v)
    assert certificate_ok(net, D)
    assert not certificate_ok(net, D + (np.arange(net.V)[:, None] == 7))   # one label off by one


def test_unreachable_or_bad_input_rejected():
    rp = np.array([0, 1, 1, 1], np.int64)              # 0 -> 1; vertex 2 unreachable
    col = np.array([1], np.int32)
    ln = np.array([5], np.int32)
    with pytest.raises(oracle.OracleError):
        oracle.road_cm(rp, col, ln, [0], [2])
    assert oracle.road_cm(rp, col, ln, [0], [1, 0]).tolist() == [[5], [0]]
    with pytest.raises(oracle.OracleError):
        oracle.road_cm(rp, np.array([3], np.int32), ln, [0], [1])      # arc to no vertex
    with pytest.raises(oracle.OracleError):
        oracle.road_cm(rp, col, np.array([-1], np.int32), [0], [1])    # negative length
