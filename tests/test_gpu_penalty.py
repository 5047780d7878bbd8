"""GPU parity with general penalty functions (Definition of the penalty
function, Section 2), given as one table per center, against the oracle.

Bit-exact: allotment, loads, the int64 objective of Equation (2) and, at
checkpoints, the whole best-transfer table.  All calls go through the C ABI.
"""
import sys

import numpy as np
import pytest

import lbdd_inputs as L
import oracle
from tests import pins
from tests.test_oracle_penalty import _cases

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


def gpu_table(lb, cm, cap, off, val, device_cm=True):
    import torch
    c = torch.from_numpy(np.ascontiguousarray(cm)).cuda() if device_cm else cm
    with lb.Instance(c, cap, pen_table=(off, val)) as I:
        I.solve()
        load, W, _ = I.snapshot()
        return I.objective(), I.assignment(), load, W, I.stats()


SMALL = _cases(60, 20000)


@pytest.mark.parametrize("case", range(60))
def test_small_tables_bit_exact(lb, case):
    inst, off, val = SMALL[case]
    say("table small", case, inst.k, inst.n, len(val))
    ref = oracle.solve_q(inst.cm, inst.cap, off, val, want_W=True)
    obj, a, load, W, st = gpu_table(lb, inst.cm, inst.cap, off, val)
    assert obj == ref.objective
    assert np.array_equal(a, ref.assign)
    assert np.array_equal(load, ref.load)
    assert np.array_equal(W, ref.W)
    assert st["cycles"] == int(ref.stats[0]) and st["paths"] == int(ref.stats[1])


@pytest.mark.parametrize("seed", range(4))
def test_table_checkpoints_bit_exact(lb, seed):
    import torch
    inst = L.random_small(k=[3, 9, 40, 70][seed], n=300, seed=40 + seed,
                          cm_hi=[5, 60, 400, 3000][seed], cap="tight", pen_hi=200)
    off, val = L.rising_penalties(inst, length=[1, 4, 40, 300][seed], seed=seed)
    say("table checkpoints", inst.name)
    with lb.Instance(torch.from_numpy(inst.cm).cuda(), inst.cap, pen_table=(off, val)) as I:
        done = 0
        for r in (1, 2, 7, 30, 64, 150, 300):
            I.solve_iters(r - done)
            done = r
            ref = oracle.solve_q(inst.cm, inst.cap, off, val, max_iters=r, want_W=True)
            load, W, _ = I.snapshot()
            assert I.objective() == ref.objective, r
            assert np.array_equal(I.assignment(), ref.assign), r
            assert np.array_equal(load, ref.load), r
            assert np.array_equal(W, ref.W), r


@pytest.mark.parametrize("k", [130, 140, 300, 1100])
def test_table_w_placement_and_wide_bit_exact(lb, k):
    inst = L.random_small(k=k, n=700 if k < 1000 else 300, seed=k, cm_hi=300, pen_hi=400)
    off, val = L.rising_penalties(inst, length=25, seed=k, step_hi=30)
    say("table wide", inst.name)
    ref = oracle.solve_q(inst.cm, inst.cap, off, val)
    obj, a, _, _, _ = gpu_table(lb, inst.cm, inst.cap, off, val)
    assert obj == ref.objective and np.array_equal(a, ref.assign)


def test_one_value_tables_equal_constant_penalties(lb):
    """A table of one value per center is the constant penalty: the GPU gives
    the same result through either entry point (C1 workload)."""
    import torch
    inst = L.make_config("C1")
    c = torch.from_numpy(inst.cm).cuda()
    with lb.Instance(c, inst.cap, inst.pen) as I:
        I.solve()
        o1, a1 = I.objective(), I.assignment()
    off = np.arange(inst.k + 1, dtype=np.int64)
    with lb.Instance(c, inst.cap, pen_table=(off, inst.pen)) as I:
        I.solve()
        assert I.objective() == o1 and np.array_equal(I.assignment(), a1)


def test_c2_workload_rising_penalties_bit_exact(lb):
    """The 100-center, 100,000-unit workload with penalties that start at the
    constant ones and rise by U{0..20} per further unit beyond capacity (2,000
    values per center): bit-exact against the oracle, and the objective is
    Equation (2) recomputed from the allotment."""
    inst = L.make_config("C2")
    off, val = L.rising_penalties(inst, length=2000, seed=2)
    say("table C2 oracle")
    ref = oracle.solve_q(inst.cm, inst.cap, off, val)
    obj, a, load, W, st = gpu_table(lb, inst.cm, inst.cap, off, val)
    say("table C2", obj, st)
    assert obj == ref.objective and np.array_equal(a, ref.assign)
    assert obj == pins.eq2(inst.cm, inst.cap, off, val, a)
    assert not pins.has_negative_cycle(W)


def test_tables_in_a_batch_and_from_host(lb):
    import torch
    insts = []
    refs = []
    for j in range(6):
        inst, off, val = SMALL[j * 7 + 3]
        refs.append(oracle.solve_q(inst.cm, inst.cap, off, val))
        c = torch.from_numpy(inst.cm).cuda() if j % 2 else inst.cm
        insts.append(lb.Instance(c, inst.cap, pen_table=(off, val)))
    lb.solve_batch(insts)
    for I, ref in zip(insts, refs):
        assert I.objective() == ref.objective and np.array_equal(I.assignment(), ref.assign)
        I.close()


def test_malformed_tables_rejected(lb):
    inst = L.random_small(k=3, n=10, seed=1)
    off = np.array([0, 1, 3, 4], np.int64)
    for val in ([5, 9, 8, 3], [5, 0, 8, 3], [5, 8, 9, 2**30]):
        with pytest.raises(lb.LbddError):
            lb.Instance(inst.cm, inst.cap, pen_table=(off, np.array(val, np.int64)))
    with pytest.raises(lb.LbddError):
        lb.Instance(inst.cm, inst.cap, pen_table=(np.array([0, 1, 1, 2], np.int64),
                                                  np.array([5, 8], np.int32)))
