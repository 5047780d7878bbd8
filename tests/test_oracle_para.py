"""The para-ASRAL-style CPU baseline (the oracle's source built with OpenMP,
Section 3.6: Gamma data-structure updates, split graphs and Bellman-Ford
rounds in threads) gives exactly the plain oracle's results.  Instances have
k >= 64 so that the threaded loops run."""
import os

import numpy as np
import pytest

import lbdd_inputs as L
import oracle


@pytest.fixture(scope="module")
def para():
    os.environ.setdefault("OMP_NUM_THREADS", "4")
    return oracle.load_para()


@pytest.mark.parametrize("k,n,seed,cap", [(64, 1500, 1, "tight"), (80, 2500, 2, "tight"),
                                           (100, 1200, 3, "zero"), (70, 3000, 4, 20)])
def test_para_equals_plain(para, k, n, seed, cap):
    inst = L.random_small(k=k, n=n, seed=seed, cm_hi=400, cap=cap, pen_hi=300)
    a = oracle.solve(*inst.arrays(), want_W=True, want_trace=True)
    b = oracle.solve(*inst.arrays(), want_W=True, want_trace=True, lib=para)
    assert a.objective == b.objective
    for x, y in ((a.assign, b.assign), (a.load, b.load), (a.W, b.W), (a.trace, b.trace), (a.stats, b.stats)):
        assert np.array_equal(x, y)


def test_para_strict_and_tables_equal_plain(para):
    inst = L.random_small(k=66, n=2000, seed=9, cm_hi=300, cap="tight", pen_hi=200)
    a = oracle.solve_strict(inst.cm, inst.cap, want_W=True)
    b = oracle.solve_strict(inst.cm, inst.cap, want_W=True, lib=para)
    assert a.objective == b.objective and np.array_equal(a.assign, b.assign) and np.array_equal(a.W, b.W)
    off, val = L.rising_penalties(inst, length=50, seed=9)
    a = oracle.solve_q(inst.cm, inst.cap, off, val)
    b = oracle.solve_q(inst.cm, inst.cap, off, val, lib=para)
    assert a.objective == b.objective and np.array_equal(a.assign, b.assign)
