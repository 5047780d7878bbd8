"""GPU parity of the road-network cost matrix (construction of CM, Section
3.5) against the oracle's Dijkstra, bit-exact, and the paper-shaped workload
end to end: the 65,902-vertex network with 131 centers, its cost matrix built
on the GPU, then solved by ASRAL and compared with the oracle.  All calls go
through the C ABI.
"""
import sys

import numpy as np
import pytest

import lbdd_inputs as L
import oracle
from tests.test_oracle_road import _random_graph

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lb():
    import torch
    import paper_2304_06543_amd.lbdd as lb
    lb.load()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lb


def gpu_cm(lb, row_ptr, col, ln, centers, units):
    import torch
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()
    cm = lb.road_cost_matrix(t(row_ptr, np.int64), t(col, np.int32), t(ln, np.int32),
                             t(centers, np.int32), t(units, np.int32))
    return cm.cpu().numpy()


@pytest.mark.parametrize("seed", range(12))
def test_small_graphs_bit_exact(lb, seed):
    rng = np.random.default_rng(seed)
    V = int(rng.integers(2, 40))
    rp, col, ln = _random_graph(rng, V, 0.15, two_way=bool(seed % 2), lmax=[2, 50, 1000][seed % 3])
    k = int(rng.integers(1, V + 1))
    centers = rng.choice(V, size=k, replace=False).astype(np.int32)
    units = rng.integers(0, V, size=int(rng.integers(1, 300))).astype(np.int32)
    say("road small", seed, V, k, len(units))
    assert np.array_equal(gpu_cm(lb, rp, col, ln, centers, units),
                          oracle.road_cm(rp, col, ln, centers, units))


@pytest.mark.parametrize("V,width,k", [(500, 20, 7), (5000, 71, 64), (20_000, 141, 300)])
def test_generated_networks_bit_exact(lb, V, width, k):
    """k = 300 runs the searches in two chunks (256 centers at a time)."""
    net = L.road_network(V, width, k, seed=V)
    say("road network", V, k)
    assert np.array_equal(gpu_cm(lb, net.row_ptr, net.col, net.length, net.centers, net.units),
                          oracle.road_cm(net.row_ptr, net.col, net.length, net.centers, net.units))


def test_r1_workload_end_to_end(lb):
    """The paper-shaped workload (65,902 vertices, 131 centers, 65,771 units,
    total capacity 0.7 n, penalties U{1..200}): cost matrix and ASRAL solve,
    both bit-exact against the oracle."""
    import torch
    net = L.make_road_config("R1")
    say("R1 oracle cost matrix")
    cm_ref = oracle.road_cm(net.row_ptr, net.col, net.length, net.centers, net.units)
    cm = gpu_cm(lb, net.row_ptr, net.col, net.length, net.centers, net.units)
    assert np.array_equal(cm, cm_ref)
    say("R1 oracle solve")
    ref = oracle.solve(cm_ref, net.cap, net.pen)
    with lb.Instance(torch.from_numpy(cm).cuda(), net.cap, net.pen) as I:
        I.solve()
        assert I.objective() == ref.objective
        assert np.array_equal(I.assignment(), ref.assign)
    say("R1", ref.objective)


def test_bad_networks_rejected(lb):
    rp = np.array([0, 1, 1, 1], np.int64)              # 0 -> 1; vertex 2 unreachable
    col = np.array([1], np.int32)
    ln = np.array([5], np.int32)
    with pytest.raises(lb.LbddError):
        gpu_cm(lb, rp, col, ln, [0], [2])
    assert gpu_cm(lb, rp, col, ln, [0], [1, 0]).tolist() == [[5], [0]]
    with pytest.raises(lb.LbddError):                  # arc to no vertex
        gpu_cm(lb, rp, np.array([3], np.int32), ln, [0], [1])
    with pytest.raises(lb.LbddError):                  # negative length
        gpu_cm(lb, rp, col, np.array([-1], np.int32), [0], [1])
    with pytest.raises(lb.LbddError):                  # decreasing offsets
        gpu_cm(lb, np.array([0, 1, 0, 1], np.int64), col, ln, [0], [1])
    with pytest.raises(lb.LbddError):                  # center outside the network
        gpu_cm(lb, rp, col, ln, [3], [1])
