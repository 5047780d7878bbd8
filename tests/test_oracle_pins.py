"""Pins of the CPU oracle against what the paper and mathematics fix.

Each check is independent of the oracle's own code: hand-worked fixtures,
brute force, an exact assignment solver (scipy), Floyd-Warshall, and the
invariants the paper proves (Lemmas 1 and 2) or that follow from its
accounting (Equation (1)).
"""
import json
import os

import numpy as np
import pytest

import lbdd_inputs as L
from tests import pins

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# --------------------------------------------------------------- setup (a1)
@pytest.mark.parametrize("seed", range(6))
def test_setup_matches_argmin_and_lexsort(orc, seed):
    """Most suitable center = first argmin (numpy); order = lexsort by (cost, id)."""
    inst = L.random_small(k=1 + seed % 5, n=300, seed=seed, cm_hi=6)
    smin, mc, order, rank = orc.setup(inst.cm)
    ref_smin = np.argmin(inst.cm, axis=1)           # first occurrence on ties
    ref_mc = inst.cm[np.arange(inst.n), ref_smin]
    ref_order = np.lexsort((np.arange(inst.n), ref_mc))
    assert np.array_equal(smin, ref_smin)
    assert np.array_equal(mc, ref_mc)
    assert np.array_equal(order, ref_order)
    assert np.array_equal(rank[order], np.arange(inst.n))


# ------------------------------------------------------------- Gamma (a3)
def test_best_transfers_hand_example(orc):
    g = _load("gamma_k3n4.json")
    cm = np.array(g["cm"], np.int32)
    W = orc.best_transfers(cm, np.array(g["assign"]), np.array(g["rank"]))
    dl, rk = pins.key_delta(W), orc.key_rank(W)
    for u in range(g["k"]):
        for v in range(g["k"]):
            exp = g["expected_delta"][u][v]
            if exp is None:
                assert W[u, v] == pins.KEY_NONE, (u, v)
            else:
                assert (dl[u, v], rk[u, v]) == (exp, g["expected_rank"][u][v]), (u, v)


def test_best_transfers_unallotted_ignored(orc):
    cm = np.array([[1, 9], [4, 0]], np.int32)
    W = orc.best_transfers(cm, np.array([-1, 1]), np.array([0, 1]))
    assert W[1, 0] != pins.KEY_NONE and pins.key_delta(W)[1, 0] == 4
    assert W[0, 1] == pins.KEY_NONE


# ----------------------------------------------- split graphs + BF (a4, a5)
def _random_W(rng, k, p_none=0.2, lo=-30, hi=30):
    """A random condensed graph with no negative cycle: deltas from potentials
    plus a nonnegative slack (reduced costs >= 0 guarantee no negative cycle)."""
    pot = rng.integers(-20, 20, size=k)
    W = np.full((k, k), pins.KEY_NONE, np.uint64)
    for u in range(k):
        for v in range(k):
            if u == v or rng.random() < p_none:
                continue
            d = int(pot[v] - pot[u] + rng.integers(0, hi))
            W[u, v] = np.uint64(((d + 2**31) << 32) | int(rng.integers(0, 1000)))
    return W


@pytest.mark.parametrize("seed", range(40))
def test_refine_search_matches_path_enumeration(orc, seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 7))
    W = _random_W(rng, k, p_none=0.3)
    anchor = int(rng.integers(0, k))
    mode = seed % 2
    load = rng.integers(0, 4, size=k).astype(np.int32)
    cap = rng.integers(0, 4, size=k).astype(np.int32)
    pen = rng.integers(1, 40, size=k).astype(np.int32)
    dist, pred, rounds = orc.refine_search(W, anchor, mode, load, cap, pen)
    E = pins.split_graph(W, anchor, mode, load, cap, pen)
    best = pins.min_simple_path(E, k, anchor)
    if best is None:
        assert dist[k] == orc.DIST_NONE
        return
    assert dist[k] == best
    # the predecessor chain is a simple path of exactly that cost
    node, cost, seen = k, 0, {k}
    while node != anchor:
        p = int(pred[node])
        assert p >= 0 and p not in seen
        cost += E[(p, node)]
        seen.add(p)
        node = p
    assert cost == best
    assert 1 <= rounds <= k + 1


def test_refine_search_reports_negative_cycle(orc):
    """A negative cycle away from the anchor is reported, not silently used."""
    k = 3
    W = np.full((k, k), pins.KEY_NONE, np.uint64)
    def key(d, r):
        return np.uint64(((d + 2**31) << 32) | r)
    W[0, 1] = key(1, 0)
    W[1, 2] = key(-5, 1)
    W[2, 1] = key(2, 2)
    with pytest.raises(orc.OracleError) as e:
        orc.refine_search(W, 0, 0, np.zeros(3, np.int32), np.zeros(3, np.int32),
                          np.ones(3, np.int32))
    assert e.value.rc == orc.E_NEGCYCLE


# ---------------------------------------------------- whole solve (a2..a7)
def test_hand_traced_run(orc):
    g = _load("asral_trace_k3n4.json")
    cm = np.array(g["cm"], np.int32)
    r = orc.solve(cm, np.array(g["cap"]), np.array(g["pen"]), want_trace=True)
    assert r.assign.tolist() == g["expected_assign"]
    assert r.objective == g["expected_objective"]
    t = g["expected_trace"]
    assert r.trace[:, 0].tolist() == t["vacant"]
    assert r.trace[:, 1].tolist() == t["cycle_cost"]
    assert r.trace[:, 3].tolist() == t["path_cost"]
    assert r.trace[:, 7].tolist() == t["objective"]


@pytest.mark.parametrize("seed", range(25))
def test_brute_force_equals_assignment_optimum(seed):
    """Pins the exact-optimum routine itself on instances small enough for k^n."""
    inst = L.random_small(k=2 + seed % 2, n=5 + seed % 3, seed=seed, cm_hi=20, pen_hi=15)
    assert pins.opt_brute(*inst.arrays()) == pins.opt_assignment(*inst.arrays())


def _cases():
    out = []
    for s in range(30):
        out.append(L.random_small(k=1 + s % 6, n=6 + (7 * s) % 40, seed=s,
                                  cm_hi=(4 if s % 3 == 0 else 60), pen_hi=(5 if s % 4 == 0 else 80)))
    return out


@pytest.mark.parametrize("inst", _cases(), ids=lambda i: i.name)
def test_solve_bounds_and_accounting(orc, inst):
    """Delta >= exact optimum; Delta = Equation (1) of the returned allotment;
    every unit allotted once; loads agree."""
    r = orc.solve(*inst.arrays(), want_trace=True)
    assert (r.assign >= 0).all() and (r.assign < inst.k).all()
    assert np.array_equal(np.bincount(r.assign, minlength=inst.k), r.load)
    assert r.objective == pins.eq1(*inst.arrays(), r.assign)
    assert r.objective >= pins.opt_assignment(*inst.arrays())


@pytest.mark.parametrize("inst", _cases()[:18], ids=lambda i: i.name)
def test_invariants_every_iteration(orc, inst):
    """After every iteration: Lemmas 1-2 (no negative cycle in Gamma), heap
    tops = definition of Gamma, Delta = Equation (1), applied refinements are
    strictly negative, the objective step matches the trace, and a center that
    has reached capacity never regains vacancy."""
    full = orc.solve(*inst.arrays(), want_trace=True)
    _, _, order, rank = orc.setup(inst.cm)
    tr = full.trace
    was_full = np.zeros(inst.k, bool)
    prev = 0
    for r in range(1, inst.n + 1):
        st = orc.solve(*inst.arrays(), max_iters=r, want_W=True)
        a = st.assign
        assert (a[order[:r]] >= 0).all() and (a[order[r:]] == -1).all()
        Wdef = orc.best_transfers(inst.cm, a, rank)
        assert np.array_equal(st.W, Wdef)
        assert not pins.has_negative_cycle(Wdef)
        assert st.objective == pins.eq1(*inst.arrays(), a)
        row = tr[r - 1]
        assert row[1] <= 0 and row[3] <= 0
        assert (row[1] == 0) == (row[2] == 0) and (row[3] == 0) == (row[4] == 0)
        d = order[r - 1]
        s = int(np.argmin(inst.cm[d]))
        step = int(inst.cm[d, s]) + (0 if row[0] else int(inst.pen[s])) + row[1] + row[3]
        assert st.objective - prev == step
        prev = st.objective
        assert not (was_full & (st.load < inst.cap)).any()
        was_full |= st.load >= inst.cap
    assert prev == full.objective


@pytest.mark.parametrize("seed", range(8))
def test_loose_capacity_gives_most_suitable(orc, seed):
    """cap >= n everywhere: nothing is ever overloaded and every transfer cost
    out of a unit's cheapest center is >= 0, so no refinement applies: the
    allotment is the row argmin and Delta = sum of row minima."""
    inst = L.random_small(k=1 + seed, n=200, seed=seed, cap="loose", cm_hi=30)
    r = orc.solve(*inst.arrays())
    assert np.array_equal(r.assign, np.argmin(inst.cm, axis=1))
    assert r.objective == int(inst.cm.min(axis=1).sum())


@pytest.mark.parametrize("seed", range(20))
def test_zero_capacity_reaches_optimum(orc, seed):
    """cap = 0 everywhere: every unit pays its center's penalty, so Equation (1)
    separates per unit and the optimum is sum_d min_s CM(d,s)+pen[s]; ASRAL's
    path refinement reaches it (checked against the exact assignment optimum
    and, when the per-unit minimum is unique, the allotment itself)."""
    inst = L.random_small(k=1 + seed % 6, n=10 + 3 * seed, seed=seed, cap="zero", cm_hi=50,
                          pen_hi=60)
    r = orc.solve(*inst.arrays())
    cmp = inst.cm.astype(np.int64) + inst.pen[None, :]
    assert r.objective == int(cmp.min(axis=1).sum())
    assert r.objective == pins.opt_assignment(*inst.arrays())
    uniq = (cmp == cmp.min(axis=1, keepdims=True)).sum(axis=1) == 1
    assert np.array_equal(r.assign[uniq], np.argmin(cmp, axis=1)[uniq])


@pytest.mark.parametrize("cap0", [0, 3, 50, 200])
def test_single_center_closed_form(orc, cap0):
    inst = L.random_small(k=1, n=120, seed=cap0, cap=cap0, cm_hi=40)
    r = orc.solve(*inst.arrays())
    assert (r.assign == 0).all()
    assert r.objective == int(inst.cm.sum()) + int(inst.pen[0]) * max(0, 120 - cap0)


def test_config_c1_accounting(orc):
    inst = L.make_config("C1")
    r = orc.solve(*inst.arrays())
    assert r.objective == pins.eq1(*inst.arrays(), r.assign)
    assert r.objective >= pins.opt_assignment(*inst.arrays())


def test_invalid_inputs_rejected(orc):
    cm = np.ones((3, 2), np.int32)
    good = (np.ones(2, np.int32), np.ones(2, np.int32))
    for bad in ([np.full((3, 2), -1, np.int32), *good],
                [np.full((3, 2), 2**30, np.int32), *good],
                [cm, np.array([-1, 1], np.int32), good[1]],
                [cm, good[0], np.array([0, 1], np.int32)]):
        with pytest.raises(orc.OracleError) as e:
            orc.solve(*bad)
        assert e.value.rc == orc.E_INVAL


# ------------------------------------------------------ Equation (1) itself
def test_objective_hand_example(orc):
    """Equation (1) worked by hand: units 0 and 1 at center 0 (capacity 1, so
    one unit beyond it pays 10), unit 2 not allotted, unit 3 at center 1 within
    capacity: 1 + 2 + 10 + 6 = 19."""
    cm = np.array([[1, 5], [2, 3], [4, 0], [9, 6]], np.int32)
    cap = np.array([1, 1], np.int32)
    pen = np.array([10, 7], np.int32)
    assert orc.objective(cm, cap, pen, np.array([0, 0, -1, 1], np.int32)) == 19
    # every unit at center 1: 5 + 3 + 0 + 6 plus three units beyond capacity at 7
    assert orc.objective(cm, cap, pen, np.array([1, 1, 1, 1], np.int32)) == 14 + 21
    # nothing allotted
    assert orc.objective(cm, cap, pen, np.full(4, -1, np.int32)) == 0


@pytest.mark.parametrize("seed", range(8))
def test_objective_matches_equation_1(orc, seed):
    """Random allotments with unallotted units, overloaded, empty and
    zero-capacity centers against the independent rendering of Equation (1)."""
    rng = np.random.default_rng(seed)
    k, n = int(rng.integers(1, 12)), int(rng.integers(1, 400))
    cm = rng.integers(0, 1 << 20, size=(n, k)).astype(np.int32)
    cap = rng.integers(0, max(2, n // k), size=k).astype(np.int32)
    pen = rng.integers(1, 1 << 20, size=k).astype(np.int32)
    assign = rng.integers(-1, k, size=n).astype(np.int32)
    load = np.bincount(assign[assign >= 0], minlength=k)
    if seed % 2 == 0:
        assert (load > cap).any()                # some center pays penalties
    assert orc.objective(cm, cap, pen, assign) == pins.eq1(cm, cap, pen, assign)


def test_objective_of_a_solve_equals_its_tracked_delta(orc):
    """The objective ASRAL tracks step by step equals Equation (1) evaluated
    on the allotment it returns."""
    inst = L.make_config("C1")
    r = orc.solve(*inst.arrays())
    assert orc.objective(*inst.arrays(), r.assign) == r.objective == pins.eq1(*inst.arrays(), r.assign)


def test_objective_rejects_unknown_center(orc):
    cm = np.ones((3, 2), np.int32)
    with pytest.raises(orc.OracleError):
        orc.objective(cm, np.ones(2, np.int32), np.ones(2, np.int32), np.array([0, 2, 1], np.int32))
