"""Pins of the oracle's general penalty functions (Definition of the penalty
function, Section 2), independent of its code.

A penalty function q_s(j) is given as a table per center whose last value
holds for every later unit.  The pins: a table of one value per center is the
constant penalty already pinned elsewhere (every output equal); extending a
table by repeating its last value changes nothing; the objective after every
iteration is Equation (2) recomputed from the allotment; it never falls below
the exact optimum, which a unit x slot assignment finds for non-decreasing
penalties (itself checked against brute force); the path search returns the
cheapest simple path of the NPath graph built here with table penalties.
"""
import itertools

import numpy as np
import pytest

import lbdd_inputs as L
import oracle
from tests import pins
from tests.test_oracle_pins import _random_W


def random_table(rng, k, maxlen, lo=1, hi=60, step=40):
    """Non-decreasing penalty tables: (off[k+1] int64, val int32)."""
    lens = rng.integers(1, maxlen + 1, size=k)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    val = []
    for s in range(k):
        v = int(rng.integers(lo, hi))
        for _ in range(int(lens[s])):
            val.append(v)
            v += int(rng.integers(0, step))
    return off, np.array(val, np.int32)


def _cases(count, seed0):
    out = []
    for j in range(count):
        rng = np.random.default_rng(seed0 + j)
        k = int(rng.integers(1, 7))
        n = int(rng.integers(1, 60))
        inst = L.random_small(k=k, n=n, seed=seed0 + j, cm_hi=[3, 40, 500][j % 3],
                              cap=["tight", "zero", 2, "loose"][j % 4])
        off, val = random_table(rng, k, [1, 3, 30][j % 3])
        out.append((inst, off, val))
    return out


@pytest.mark.parametrize("j", range(30))
def test_one_value_per_center_is_the_constant_penalty(j):
    inst = L.random_small(k=1 + j % 8, n=20 + 7 * j, seed=900 + j, cm_hi=[3, 50, 400][j % 3],
                          cap=["tight", "zero", 3][j % 3], pen_hi=[5, 90, 700][j % 3])
    off = np.arange(inst.k + 1, dtype=np.int64)
    a = oracle.solve(*inst.arrays(), want_W=True, want_trace=True)
    b = oracle.solve_q(inst.cm, inst.cap, off, inst.pen, want_W=True, want_trace=True)
    assert a.objective == b.objective
    for x, y in ((a.assign, b.assign), (a.load, b.load), (a.W, b.W), (a.trace, b.trace),
                 (a.stats, b.stats)):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("j", range(10))
def test_repeating_the_last_value_changes_nothing(j):
    inst, off, val = _cases(10, 3100)[j]
    lens = np.diff(off)
    ext = []
    for s in range(inst.k):
        t = list(val[off[s]:off[s + 1]])
        ext.append(t + [t[-1]] * (j + 1))
    off2 = np.concatenate([[0], np.cumsum([len(t) for t in ext])]).astype(np.int64)
    val2 = np.array([x for t in ext for x in t], np.int32)
    a = oracle.solve_q(inst.cm, inst.cap, off, val, want_W=True)
    b = oracle.solve_q(inst.cm, inst.cap, off2, val2, want_W=True)
    assert lens.sum() < len(val2)
    assert a.objective == b.objective and np.array_equal(a.assign, b.assign)
    assert np.array_equal(a.W, b.W)


@pytest.mark.parametrize("j", range(24))
def test_objective_is_equation2_after_every_iteration(j):
    inst, off, val = _cases(24, 4200)[j]
    for r in range(1, inst.n + 1):
        st = oracle.solve_q(inst.cm, inst.cap, off, val, max_iters=r, want_W=True)
        assert st.objective == pins.eq2(inst.cm, inst.cap, off, val, st.assign), r
        assert not pins.has_negative_cycle(st.W), r
        assert np.array_equal(np.bincount(st.assign[st.assign >= 0], minlength=inst.k), st.load)


@pytest.mark.parametrize("j", range(24))
def test_objective_at_least_the_convex_optimum(j):
    inst, off, val = _cases(24, 5300)[j]
    r = oracle.solve_q(inst.cm, inst.cap, off, val)
    assert r.objective >= pins.opt_convex(inst.cm, inst.cap, off, val)


@pytest.mark.parametrize("seed", range(12))
def test_convex_optimum_equals_brute_force(seed):
    """The slot expansion behind opt_convex, against enumeration of all k^n
    allotments under Equation (2)."""
    rng = np.random.default_rng(seed)
    k, n = int(rng.integers(1, 4)), int(rng.integers(1, 7))
    cm = rng.integers(0, 30, size=(n, k)).astype(np.int32)
    cap = rng.integers(0, 3, size=k).astype(np.int32)
    off, val = random_table(rng, k, 4, step=25)
    best = min(pins.eq2(cm, cap, off, val, np.array(a))
               for a in itertools.product(range(k), repeat=n))
    assert pins.opt_convex(cm, cap, off, val) == best


@pytest.mark.parametrize("seed", range(16))
def test_path_search_with_table_penalties(seed):
    """NPath with table penalties: the edge u -> s*_in costs what one more unit
    at u would pay minus what the anchor's last unit beyond capacity pays."""
    rng = np.random.default_rng(600 + seed)
    k = int(rng.integers(2, 6))
    W = _random_W(rng, k, p_none=0.2)
    cap = rng.integers(0, 4, size=k).astype(np.int32)
    load = rng.integers(0, 8, size=k).astype(np.int32)
    a = int(rng.integers(0, k))
    load[a] = cap[a] + int(rng.integers(1, 4))          # the anchor is overloaded
    off, val = random_table(rng, k, 5)
    E = {}
    dl = pins.key_delta(W)
    for u in range(k):
        for v in range(k):
            if u != v and v != a and W[u, v] != pins.KEY_NONE:
                E[(u, v)] = int(dl[u, v])
    q_anchor = pins.table_penalty(off, val, a, int(load[a] - cap[a]))
    for u in range(k):
        if u != a:
            qu = pins.table_penalty(off, val, u, int(load[u] - cap[u] + 1)) if load[u] >= cap[u] else 0
            E[(u, k)] = qu - q_anchor
    dist, pred, _ = oracle.refine_search_q(W, a, 1, load, cap, off, val)
    best = pins.min_simple_path(E, k, a)
    if best is None:
        assert dist[k] == oracle.DIST_NONE
    else:
        assert dist[k] == best


def test_rejects_bad_tables():
    inst = L.random_small(k=3, n=10, seed=1)
    good_off = np.array([0, 1, 3, 4], np.int64)
    with pytest.raises(oracle.OracleError):       # decreasing
        oracle.solve_q(inst.cm, inst.cap, good_off, np.array([5, 9, 8, 3], np.int32))
    with pytest.raises(oracle.OracleError):       # zero penalty
        oracle.solve_q(inst.cm, inst.cap, good_off, np.array([5, 0, 8, 3], np.int32))
    with pytest.raises(oracle.OracleError):       # a center without values
        oracle.solve_q(inst.cm, inst.cap, np.array([0, 1, 1, 2], np.int64),
                       np.array([5, 8], np.int32))
