"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU,
in a temporary directory), builds it, and runs a quick subset of the pins:
at least one must fail.  Mistakes that only change which of several equally
cheap answers is returned (tie rules, applying zero-cost refinements) are not
listed: the paper leaves those open and no pin can see them.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import lbdd_inputs as L
import oracle
from tests import pins
from tests.test_oracle_pins import _load, _random_W

MUTANTS = {
    "transfer_cost_sign": ("(int64_t)row[v] - row[u], S->rank[d]", "(int64_t)row[u] - row[v], S->rank[d]"),
    "no_penalty_on_overload": ("delta += (int64_t)cm[d * (int64_t)k + s] + q;",
                               "delta += (int64_t)cm[d * (int64_t)k + s];"),
    "penalty_edge_ignores_load": ("wt[(int64_t)u * K1 + k] = q_next(P, load, cap, u) - q_last(P, load, cap, anchor);",
                                  "wt[(int64_t)u * K1 + k] = q_at(P, u, 1) - q_last(P, load, cap, anchor);"),
    "q_next_first_value_only": ("return load[u] >= cap[u] ? q_at(P, u, (int64_t)load[u] - cap[u] + 1) : 0;",
                                "return load[u] >= cap[u] ? q_at(P, u, 1) : 0;"),
    "q_last_off_by_one": ("q_at(P, u, load[u] > cap[u] ? (int64_t)load[u] - cap[u] : 1);",
                          "q_at(P, u, load[u] > cap[u] ? (int64_t)load[u] - cap[u] + 1 : 1);"),
    "q_table_tail_uses_first_value": ("(j < len ? j : len) - 1]", "(j < len ? j : 1) - 1]"),
    "road_skips_last_arc": ("for (int64_t i = row_ptr[x.v]; i < row_ptr[x.v + 1]; ++i) {",
                            "for (int64_t i = row_ptr[x.v]; i + 1 < row_ptr[x.v + 1]; ++i) {"),
    "road_settled_entries_skipped": ("if (x.d > dist[x.v]) continue;",
                                     "if (x.d >= dist[x.v] && x.d > 0) continue;"),
    "vacancy_off_by_one": ("int vacant = S.load[s] < cap[s];", "int vacant = S.load[s] <= cap[s];"),
    "no_path_refinement": ("if (!vacant) {", "if (0) {"),
    "no_cycle_refinement": ("rc = refine(&S, s, 0, &cyc_cost", "if (0) rc = refine(&S, s, 0, &cyc_cost"),
    "stale_heap_tops": ("if (S->a[d] == u) return key;", "return key;"),
    "last_argmin": ("if (row[s] < row[best]) best = s;", "if (row[s] <= row[best]) best = s;"),
    "order_descending": ("return x->mc < y->mc ? -1 : 1;", "return x->mc < y->mc ? 1 : -1;"),
    "transposed_gamma_edge": ("uint64_t key = W[(int64_t)u * k + v];\n            if (key == KEY_NONE) continue;\n            wt",
                              "uint64_t key = W[(int64_t)v * k + u];\n            if (key == KEY_NONE) continue;\n            wt"),
    "cycle_in_edge_reversed": ("uint64_t key = W[(int64_t)u * k + anchor];", "uint64_t key = W[(int64_t)anchor * k + u];"),
    "bf_stops_early": ("for (int32_t t = 1; t <= K1; ++t) {", "for (int32_t t = 1; t <= 2; ++t) {"),
    "strict_no_dummy_edges": ("if (S->strict && u != v", "if (0 && u != v"),
    "strict_allot_ignores_capacity": ("if (S.load[t] < capx[t] && (s < 0", "if ((s < 0"),
    "strict_dummy_cost_not_above_max": ("cmx[d * kx + k] = maxcm + 1;", "cmx[d * kx + k] = maxcm;"),
    "objective_penalty_on_whole_load": ("total += (int64_t)pen[s] * (load[s] - cap[s]);",
                                        "total += (int64_t)pen[s] * load[s];"),
    "objective_counts_unallotted": ("        if (s < 0) continue;\n        if (s >= k) { free(load); return ORC_E_INVAL; }",
                                    "        if (s < 0) s = 0;\n        if (s >= k) { free(load); return ORC_E_INVAL; }"),
}


def _pin_failures(lib):
    """Run a quick subset of the pins against a built oracle library."""
    fails = []

    def check(name, fn):
        try:
            if not fn():
                fails.append(name)
        except Exception as e:                     # an error is a failed pin too
            fails.append(f"{name}: {type(e).__name__}")

    def setup_ok():
        inst = L.random_small(k=4, n=200, seed=3, cm_hi=6)
        smin, mc, order, _ = oracle.setup(inst.cm, lib=lib)
        return (np.array_equal(smin, np.argmin(inst.cm, 1))
                and np.array_equal(order, np.lexsort((np.arange(inst.n), inst.cm.min(1)))))

    def hand_trace_ok():
        g = _load("asral_trace_k3n4.json")
        r = oracle.solve(np.array(g["cm"], np.int32), np.array(g["cap"]), np.array(g["pen"]), lib=lib)
        return r.assign.tolist() == g["expected_assign"] and r.objective == g["expected_objective"]

    def search_ok():
        for seed in range(12):
            rng = np.random.default_rng(seed)
            k = int(rng.integers(2, 6))
            W = _random_W(rng, k, p_none=0.2)
            load = rng.integers(0, 4, size=k).astype(np.int32)
            cap = rng.integers(0, 4, size=k).astype(np.int32)
            pen = rng.integers(1, 40, size=k).astype(np.int32)
            a = int(rng.integers(0, k))
            dist, _, _ = oracle.refine_search(W, a, seed % 2, load, cap, pen, lib=lib)
            best = pins.min_simple_path(pins.split_graph(W, a, seed % 2, load, cap, pen), k, a)
            if (best is None) != (dist[k] == oracle.DIST_NONE) or (best is not None and dist[k] != best):
                return False
        return True

    def solve_ok():
        for s in range(8):
            inst = L.random_small(k=2 + s % 4, n=25, seed=s, cm_hi=40, pen_hi=60)
            _, _, order, rank = oracle.setup(inst.cm, lib=lib)
            for r in (5, 12, 25):
                st = oracle.solve(*inst.arrays(), max_iters=r, want_W=True, lib=lib)
                Wdef = oracle.best_transfers(inst.cm, st.assign, rank, lib=lib)
                if (not np.array_equal(st.W, Wdef) or pins.has_negative_cycle(Wdef)
                        or st.objective != pins.eq1(*inst.arrays(), st.assign)):
                    return False
            if st.objective < pins.opt_assignment(*inst.arrays()):
                return False
        return True

    def zero_cap_ok():
        for s in range(6):
            inst = L.random_small(k=2 + s % 4, n=20, seed=s, cap="zero", cm_hi=50, pen_hi=60)
            r = oracle.solve(*inst.arrays(), lib=lib)
            if r.objective != int((inst.cm.astype(np.int64) + inst.pen).min(1).sum()):
                return False
        return True

    def strict_ok():
        for s in range(10):
            rng = np.random.default_rng(900 + s)
            k, n = 2 + s % 4, 30
            cm = rng.integers(0, 30, size=(n, k)).astype(np.int32)
            cap = rng.integers(0, 2 * n // k, size=k).astype(np.int32)
            r = oracle.solve_strict(cm, cap, lib=lib)
            real = r.assign >= 0
            if (np.bincount(r.assign[real], minlength=k) > cap).any():
                return False
            if r.objective != pins.opt_strict(cm, cap):
                return False
        return True

    def table_ok():
        from tests.test_oracle_penalty import random_table
        for s in range(8):
            inst = L.random_small(k=2 + s % 4, n=30, seed=70 + s, cm_hi=40, cap="tight")
            off, val = random_table(np.random.default_rng(s), inst.k, 12)
            for r in (10, 30):
                st = oracle.solve_q(inst.cm, inst.cap, off, val, max_iters=r, want_trace=True, lib=lib)
                if st.objective != pins.eq2(inst.cm, inst.cap, off, val, st.assign):
                    return False
        return True

    def road_ok():
        from scipy.sparse import csr_matrix
        from scipy.sparse.csgraph import dijkstra
        for s in range(3):
            net = L.road_network(600 + 11 * s, 25, 6, seed=s)
            cm = oracle.road_cm(net.row_ptr, net.col, net.length, net.centers, net.units, lib=lib)
            G = csr_matrix((net.length.astype(np.float64), net.col, net.row_ptr), shape=(net.V, net.V))
            if not np.array_equal(cm, dijkstra(G, indices=net.centers)[:, net.units].T.astype(np.int64)):
                return False
        return True

    def objective_ok():
        for s in range(6):
            rng = np.random.default_rng(40 + s)
            k, n = 2 + s % 4, 60
            cm = rng.integers(0, 100, size=(n, k)).astype(np.int32)
            cap = rng.integers(0, n // k, size=k).astype(np.int32)
            pen = rng.integers(1, 50, size=k).astype(np.int32)
            a = rng.integers(-1, k, size=n).astype(np.int32)
            if oracle.objective(cm, cap, pen, a, lib=lib) != pins.eq1(cm, cap, pen, a):
                return False
        return True

    for name, fn in [("setup", setup_ok), ("objective", objective_ok), ("hand_trace", hand_trace_ok), ("search", search_ok),
                     ("solve", solve_ok), ("zero_cap", zero_cap_ok), ("strict", strict_ok),
                     ("table", table_ok), ("road", road_ok)]:
        check(name, fn)
    return fails


def test_unmutated_oracle_passes_quick_pins():
    assert _pin_failures(oracle._load()) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    with open(oracle.SRC) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation site for {name} not unique/absent"
    path = tmp_path / "mut.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / f"mut_{name}.so")
    oracle.build(src=str(path), out=so)
    # a planted mistake may also crash the library: run the pins in a child
    # process and count a crash as a failed pin
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys, oracle; from tests.test_oracle_mutants import _pin_failures; "
            f"f = _pin_failures(oracle._load({so!r})); print(f); sys.exit(3 if f else 0)")
    p = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=300)
    assert p.returncode != 0, f"mutant {name} passed every pin: {p.stdout}"
