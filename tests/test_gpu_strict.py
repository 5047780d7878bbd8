"""GPU parity of strict-LBDD (Appendix B, Algorithm 4) against the oracle.

Bit-exact like the ASRAL tests: allotment (with -1 for units left at the
dummy center), loads, the int64 objective of Equation (3) and, at
checkpoints, the whole best-transfer table with its dummy transfers.  At the
full workload sizes Theorem 2's certificate is checked as well: no negative
cycle in the final table.  All calls go through the C ABI.
"""
import sys

import numpy as np
import pytest

import lbdd_inputs as L
import oracle
from tests import pins
from tests.test_oracle_strict import _instances

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


def gpu_strict(lb, cm, cap, device_cm=True):
    import torch
    c = torch.from_numpy(np.ascontiguousarray(cm)).cuda() if device_cm else cm
    with lb.Instance(c, cap, strict=True) as I:
        I.solve()
        load, W, _ = I.snapshot()
        return I.objective(), I.assignment(), load, W, I.stats(), I.k_graph


def _check_against_oracle(lb, cm, cap, want_opt=False):
    ref = oracle.solve_strict(cm, cap, want_W=True)
    obj, a, load, W, st, kg = gpu_strict(lb, cm, cap)
    assert kg == ref.kx
    assert obj == ref.objective
    assert np.array_equal(a, ref.assign)
    assert np.array_equal(load, ref.load)
    assert np.array_equal(W, ref.W)
    assert st["cycles"] == int(ref.stats[0]) and st["paths"] == 0
    if want_opt:
        assert obj == pins.opt_strict(cm, cap)
    return st, ref


SMALL = _instances(48, 12000, (1, 400), (1, 34))


@pytest.mark.parametrize("case", range(48))
def test_small_strict_bit_exact(lb, case):
    cm, cap = SMALL[case]
    say("strict small", case, cm.shape, int(cap.sum()))
    _check_against_oracle(lb, cm, cap, want_opt=cm.shape[0] <= 150)


@pytest.mark.parametrize("seed", range(4))
def test_strict_checkpoints_bit_exact(lb, seed):
    import torch
    rng = np.random.default_rng(300 + seed)
    k, n = [3, 9, 40, 70][seed], 260
    cm = rng.integers(0, [5, 60, 400, 3000][seed], size=(n, k)).astype(np.int32)
    cap = rng.integers(0, 2 * n // k, size=k).astype(np.int32)
    say("strict checkpoints", k, n, int(cap.sum()))
    with lb.Instance(torch.from_numpy(cm).cuda(), cap, strict=True) as I:
        done = 0
        for r in (1, 2, 7, 30, 64, 150, 260):
            I.solve_iters(r - done)
            done = r
            ref = oracle.solve_strict(cm, cap, max_iters=r, want_W=True)
            load, W, _ = I.snapshot()
            assert I.objective() == ref.objective, r
            assert np.array_equal(I.assignment(), ref.assign), r
            assert np.array_equal(load, ref.load), r
            assert np.array_equal(W, ref.W), r


@pytest.mark.parametrize("k", [129, 134, 140, 300, 1100])
def test_strict_w_placement_and_wide_bit_exact(lb, k):
    """W in LDS and in global memory, and more centers than threads, with the
    dummy center added (k + 1 graph centers)."""
    rng = np.random.default_rng(k)
    n = 700 if k < 1000 else 300
    cm = rng.integers(0, 500, size=(n, k)).astype(np.int32)
    cap = rng.integers(0, max(2, 2 * n // k), size=k).astype(np.int32)
    cap[: k // 3] = 0
    say("strict wide", k, n, int(cap.sum()))
    _check_against_oracle(lb, cm, cap)


def test_strict_without_excess_demand(lb):
    """Total capacity >= n: no dummy center, dummy units only."""
    rng = np.random.default_rng(77)
    cm = rng.integers(0, 50, size=(900, 12)).astype(np.int32)
    cap = np.full(12, 80, np.int32)
    st, _ = _check_against_oracle(lb, cm, cap, want_opt=True)
    say("strict no excess", st["cycles"])


def test_strict_c1_workload_optimal(lb):
    """The 8-center, 2,000-unit workload (capacities 90 % of the demand):
    bit-exact against the oracle and equal to the assignment optimum."""
    inst = L.make_config("C1")
    st, _ = _check_against_oracle(lb, inst.cm, inst.cap, want_opt=True)
    say("strict C1", st)


def test_strict_c2_workload_bit_exact_and_certified(lb):
    """The 100-center, 100,000-unit workload (capacities 95 % of the demand,
    so 5,000 units stay unallotted): bit-exact against the oracle, and the
    final table has no negative cycle, which by Theorem 2 makes the allotment
    optimal."""
    inst = L.make_config("C2")
    say("strict C2 oracle")
    st, ref = _check_against_oracle(lb, inst.cm, inst.cap)
    say("strict C2", st)
    assert not pins.has_negative_cycle(ref.W)
    a = ref.assign
    assert int((a < 0).sum()) == inst.n - int(inst.cap.sum())
    assert (np.bincount(a[a >= 0], minlength=inst.k) <= inst.cap).all()


def test_strict_host_input_and_batch_agree(lb):
    """Host-memory CM, and strict and penalty instances mixed in one batch."""
    import torch
    rng = np.random.default_rng(5)
    items = []
    for j in range(6):
        k, n = [4, 30, 150][j % 3], 500 + 100 * j
        cm = rng.integers(0, 300, size=(n, k)).astype(np.int32)
        cap = rng.integers(0, 2 * n // k, size=k).astype(np.int32)
        items.append((cm, cap, rng.integers(1, 200, size=k).astype(np.int32)))
    solo = [gpu_strict(lb, cm, cap, device_cm=False) for cm, cap, _ in items]
    insts = []
    for j, (cm, cap, pen) in enumerate(items):
        c = torch.from_numpy(cm).cuda()
        insts.append(lb.Instance(c, cap, strict=True))
        insts.append(lb.Instance(c, cap, pen))
    lb.solve_batch(insts)
    for j, (cm, cap, pen) in enumerate(items):
        assert insts[2 * j].objective() == solo[j][0]
        assert np.array_equal(insts[2 * j].assignment(), solo[j][1])
        ref = oracle.solve(cm, cap, pen)
        assert insts[2 * j + 1].objective() == ref.objective
        assert np.array_equal(insts[2 * j + 1].assignment(), ref.assign)
    for I in insts:
        I.close()


def test_strict_rejects_what_it_cannot_hold(lb):
    import torch
    cm = np.zeros((10, 3), np.int32)
    cm[0, 0] = 2**30 - 1                       # the dummy center would cost 2^30
    with pytest.raises(lb.LbddError):
        lb.Instance(torch.from_numpy(cm).cuda(), np.array([1, 1, 1], np.int32), strict=True)
    # with room for every unit no dummy center is needed and the entry is fine
    with lb.Instance(torch.from_numpy(cm).cuda(), np.array([4, 4, 4], np.int32), strict=True) as I:
        assert I.k_graph == 3
    with pytest.raises(lb.LbddError):         # k + 1 would exceed the center limit
        lb.Instance(np.zeros((3, 2048), np.int32), np.zeros(2048, np.int32), strict=True)
    with pytest.raises(ValueError):
        lb.Instance(cm, np.ones(3, np.int32), np.ones(3, np.int32), strict=True)
