"""Pins of the strict-LBDD oracle (Appendix B, Algorithm 4), independent of
its code.  Theorem 2 makes the algorithm exact, so its objective must equal
the optimum found by other means: brute force on tiny instances, scipy's
assignment solver on a unit x (capacity slot) expansion on larger ones.  At
any size the final table (dummy transfers included) has no negative cycle,
which by Theorem 2 certifies optimality."""
import numpy as np
import pytest

import lbdd_inputs as L
import oracle
from tests import pins


def _instances(count, seed0, n_range, k_range, cm_hi_choices=(3, 50, 1000)):
    out = []
    for j in range(count):
        rng = np.random.default_rng(seed0 + j)
        k = int(rng.integers(*k_range))
        n = int(rng.integers(*n_range))
        cm = rng.integers(0, int(rng.choice(cm_hi_choices)) + 1, size=(n, k)).astype(np.int32)
        mode = j % 4
        if mode == 0:      # room for everyone
            cap = rng.integers(n // k + 1, n + 2, size=k)
        elif mode == 1:    # excess demand: a dummy center takes the rest
            cap = rng.integers(0, max(1, n // k), size=k)
        elif mode == 2:    # total capacity exactly n
            cap = np.full(k, n // k)
            cap[: n - int(cap.sum())] += 1
        else:              # some centers closed
            cap = rng.integers(0, 2 * (n // k) + 2, size=k)
            cap[rng.integers(0, k)] = 0
        out.append((cm, cap.astype(np.int32)))
    return out


def _check_invariants(cm, cap, r):
    n, k = cm.shape
    a = r.assign
    real = a >= 0
    counts = np.bincount(a[real], minlength=k)
    assert (counts <= cap).all()
    assert int((~real).sum()) == max(0, n - int(cap.sum()))
    assert r.objective == int(cm[np.arange(n)[real], a[real]].astype(np.int64).sum())


@pytest.mark.parametrize("cm,cap", _instances(40, 7000, (1, 8), (1, 4), (3, 20)))
def test_strict_equals_brute_force(cm, cap):
    r = oracle.solve_strict(cm, cap)
    _check_invariants(cm, cap, r)
    assert r.objective == pins.strict_brute(cm, cap)


@pytest.mark.parametrize("cm,cap", _instances(60, 8000, (1, 120), (1, 9)))
def test_strict_equals_assignment_optimum(cm, cap):
    r = oracle.solve_strict(cm, cap, want_W=True)
    _check_invariants(cm, cap, r)
    assert r.objective == pins.opt_strict(cm, cap)
    assert not pins.has_negative_cycle(r.W)


def test_strict_optimum_at_c1_size():
    """The 8-center, 2,000-unit workload with capacities cut to 60 % of the
    demand (so the dummy center takes 800 units)."""
    inst = L.make_config("C1")
    cap = np.full(inst.k, int(0.6 * inst.n) // inst.k, np.int32)
    r = oracle.solve_strict(inst.cm, cap, want_W=True)
    _check_invariants(inst.cm, cap, r)
    assert r.kx == inst.k + 1
    assert r.objective == pins.opt_strict(inst.cm, cap)
    assert not pins.has_negative_cycle(r.W)
    r2 = oracle.solve_strict(inst.cm, inst.cap, want_W=True)   # total 0.9 n as well
    assert r2.objective == pins.opt_strict(inst.cm, inst.cap)


def test_strict_without_capacity_pressure_is_row_argmin():
    """With room for every unit at its cheapest center nothing ever moves."""
    inst = L.random_small(k=6, n=300, seed=5, cm_hi=100)
    cap = np.full(6, 300, np.int32)
    r = oracle.solve_strict(inst.cm, cap)
    assert np.array_equal(r.assign, np.argmin(inst.cm, axis=1))
    assert r.stats[0] == 0                       # no cycle applied


def test_strict_dummy_key_orders_after_real_keys_of_equal_cost():
    """The reading for ties: a dummy transfer (cost 0) sorts after any real
    transfer of cost 0 and before any real transfer of cost 1."""
    zero_real = np.uint64((1 << 63) | 12345)               # cost 0, rank 12345
    one_real = np.uint64(((2**31 + 1) << 32) | 0)           # cost 1, rank 0
    assert zero_real < oracle.DUMMY_KEY < one_real
    assert int(oracle.key_delta(np.array([oracle.DUMMY_KEY]))[0]) == 0


@pytest.mark.parametrize("seed", range(8))
def test_strict_no_negative_cycle_after_every_iteration(seed):
    """Lemma 2 carried to strict-LBDD: each allotment lowers only the anchor's
    row, so one Negative Cycle Refinement from it leaves no negative cycle.
    Checked after every iteration of a small run, and the objective of every
    prefix is the optimum of the units allotted so far (Theorem 2 on the
    prefix: the same capacities, the first r units of the order)."""
    rng = np.random.default_rng(40 + seed)
    k, n = 2 + seed % 5, 24
    cm = rng.integers(0, [4, 30, 200][seed % 3], size=(n, k)).astype(np.int32)
    cap = rng.integers(0, 2 * n // k, size=k).astype(np.int32)
    _, _, order, _ = oracle.setup(cm)
    for r in range(1, n + 1):
        res = oracle.solve_strict(cm, cap, max_iters=r, want_W=True)
        assert not pins.has_negative_cycle(res.W), r
        sub = cm[order[:r]]
        if int(cap.sum()) >= r:
            assert res.objective == pins.opt_strict(sub, cap), r
