"""GPU parity: the HIP path against the CPU oracle, bit-exact.

Everything compared here is integer: the processing order, the allotment, the
loads, the int64 objective and the uint64 best-transfer keys.  The tie rules
of both sides are the same readings of the paper, so equality is exact.
All calls go through the C ABI (paper_2304_06543_amd.lbdd is ctypes only).
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import lbdd_inputs as L
import oracle
from tests import pins

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "oracle_results.json")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lb():
    import torch
    import paper_2304_06543_amd.lbdd as lb
    lb.load()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lb


def gpu_solve(lb, inst, device_cm=True):
    import torch
    cm = torch.from_numpy(inst.cm).cuda() if device_cm else inst.cm
    with lb.Instance(cm, inst.cap, inst.pen) as I:
        I.solve()
        return I.objective(), I.assignment(), I.stats()


def small_cases():
    out = []
    caps = ["tight", "loose", "zero", 2, "tight"]
    for s in range(60):
        k = [1, 2, 3, 4, 5, 7, 8, 12, 16, 33][s % 10]
        n = [1, 2, 9, 40, 130, 257, 400][s % 7]
        out.append(L.random_small(k=k, n=n, seed=100 + s, cm_hi=[3, 50, 1000][s % 3],
                                  cap=caps[s % 5], pen_hi=[5, 80, 600][s % 3]))
    return out


def test_processing_order_matches_oracle(lb):
    import torch
    for inst in [L.make_config("C1"), L.random_small(k=5, n=3000, seed=1, cm_hi=3)]:
        say("order", inst.name)
        _, _, order, _ = oracle.setup(inst.cm)
        with lb.Instance(torch.from_numpy(inst.cm).cuda(), inst.cap, inst.pen) as I:
            _, _, g_order = I.snapshot()
        assert np.array_equal(g_order, order)


@pytest.mark.parametrize("inst", small_cases(), ids=lambda i: i.name)
def test_small_instances_bit_exact(lb, inst):
    say("small", inst.name)
    ref = oracle.solve(*inst.arrays())
    obj, a, _ = gpu_solve(lb, inst)
    assert obj == ref.objective
    assert np.array_equal(a, ref.assign)


@pytest.mark.parametrize("seed", range(6))
def test_checkpoints_state_bit_exact(lb, seed):
    """Allotment, loads, objective and the whole best-transfer table after
    several intermediate iteration counts."""
    import torch
    inst = L.random_small(k=[3, 6, 9, 17, 40, 70][seed], n=220, seed=500 + seed,
                          cm_hi=[4, 60, 300][seed % 3], pen_hi=90)
    say("checkpoints", inst.name)
    with lb.Instance(torch.from_numpy(inst.cm).cuda(), inst.cap, inst.pen) as I:
        done = 0
        for r in (1, 2, 7, 30, 64, 150, 220):
            I.solve_iters(r - done)
            done = r
            assert I.progress() == r
            ref = oracle.solve(*inst.arrays(), max_iters=r, want_W=True)
            load, W, _ = I.snapshot()
            assert I.objective() == ref.objective, r
            assert np.array_equal(I.assignment(), ref.assign), r
            assert np.array_equal(load, ref.load), r
            assert np.array_equal(W, ref.W), r


@pytest.mark.parametrize("k", [130, 140, 300])
def test_w_placement_boundaries_bit_exact(lb, k):
    """W in LDS (k <= ~135) and in global memory give the same results."""
    inst = L.random_small(k=k, n=700, seed=k, cm_hi=200, pen_hi=300)
    say("k-boundary", inst.name)
    ref = oracle.solve(*inst.arrays())
    obj, a, _ = gpu_solve(lb, inst)
    assert obj == ref.objective and np.array_equal(a, ref.assign)


def test_more_centers_than_threads_bit_exact(lb):
    inst = L.random_small(k=1100, n=260, seed=11, cm_hi=500, cap=0, pen_hi=400)
    say("k>1024", inst.name)
    ref = oracle.solve(*inst.arrays())
    obj, a, _ = gpu_solve(lb, inst)
    assert obj == ref.objective and np.array_equal(a, ref.assign)


def test_host_and_device_inputs_agree(lb):
    inst = L.make_config("C1")
    a1 = gpu_solve(lb, inst, device_cm=True)
    a2 = gpu_solve(lb, inst, device_cm=False)
    assert a1[0] == a2[0] and np.array_equal(a1[1], a2[1])


def test_config_c1_bit_exact(lb):
    inst = L.make_config("C1")
    ref = oracle.solve(*inst.arrays())
    obj, a, st = gpu_solve(lb, inst)
    say("C1", obj, st)
    assert obj == ref.objective and np.array_equal(a, ref.assign)
    assert obj == pins.eq1(*inst.arrays(), a)


def _golden(name):
    with open(GOLD) as f:
        return json.load(f)[name]


def test_config_c2_bit_exact_against_stored_oracle(lb):
    g = _golden("C2")
    inst = L.make_config("C2")
    assert L.input_hash(inst) == g["input_sha256"], "generator produced different inputs"
    obj, a, st = gpu_solve(lb, inst)
    say("C2", obj, st)
    assert obj == g["objective"]
    assert hashlib.sha256(a.astype("<i4").tobytes()).hexdigest() == g["assignment_sha256"]
    assert obj == pins.eq1(*inst.arrays(), a)


def test_every_search_kind_runs_bit_exact(lb):
    """The solver answers a refinement search in one of several exact ways:
    Bellman-Ford rounds (pruned by the node potentials when they are
    feasible), bounded Dijkstra order on feasible node potentials (repaired
    after refinements where needed), or no search at all when the potentials
    certify there is no negative cycle.  These instances use every one of
    them, and the results still equal the oracle's.  (Answering a path search
    from the labels of an unpruned cycle search that applied nothing needs
    potentials that failed to repair, which these instances do not reach.)"""
    seen = {}
    for seed, k in ((41, 12), (42, 40), (43, 100)):
        inst = L.random_small(k=k, n=4000, seed=seed, cm_hi=300, pen_hi=400)
        say("search kinds", inst.name)
        ref = oracle.solve(*inst.arrays())
        obj, a, st = gpu_solve(lb, inst)
        assert obj == ref.objective and np.array_equal(a, ref.assign)
        for key in ("bf_rounds", "dijkstra", "potentials_kept",
                    "potential_repairs", "cycle_searches_skipped", "cycles", "paths"):
            seen[key] = seen.get(key, 0) + st[key]
    say("search kinds", seen)
    assert all(v > 0 for v in seen.values()), seen


def test_solve_is_deterministic(lb):
    inst = L.random_small(k=24, n=5000, seed=3, cm_hi=40, pen_hi=200)
    r1 = gpu_solve(lb, inst)
    r2 = gpu_solve(lb, inst)
    assert r1[0] == r2[0] and np.array_equal(r1[1], r2[1])


def test_invalid_cost_rejected(lb):
    import torch
    cm = np.ones((50, 4), np.int32)
    cm[17, 2] = -3
    with pytest.raises(lb.LbddError) as e:
        lb.Instance(torch.from_numpy(cm).cuda(), np.ones(4), np.ones(4))
    assert e.value.code == lb.E_INVAL
    cm[17, 2] = 1 << 30
    with pytest.raises(lb.LbddError):
        lb.Instance(cm, np.ones(4), np.ones(4))
    with pytest.raises(lb.LbddError):
        lb.Instance(np.ones((5, 3), np.int32), np.array([1, -1, 1]), np.ones(3))
    with pytest.raises(lb.LbddError):
        lb.Instance(np.ones((5, 3), np.int32), np.ones(3), np.array([1, 0, 1]))


# ------------------------------------------------ whole-matrix scan (a3)
@pytest.mark.parametrize("k,n", [(1, 10), (8, 2000), (37, 5000), (100, 100_000), (131, 20_000)])
def test_full_scan_bit_exact(lb, k, n):
    import torch
    rng = np.random.default_rng(k * 7 + n)
    cm = rng.integers(0, 2000, size=(n, k), dtype=np.int64).astype(np.int32)
    assign = rng.integers(-1, k, size=n).astype(np.int32)
    rank = rng.permutation(n).astype(np.int32)
    say("scan", k, n)
    ref = oracle.best_transfers(cm, assign, rank.astype(np.int64))
    cmd = torch.from_numpy(cm).cuda()
    ad, rd = torch.from_numpy(assign).cuda(), torch.from_numpy(rank).cuda()
    work = torch.empty(lb.best_transfers_work_bytes(k, n), dtype=torch.uint8, device="cuda")
    W = lb.best_transfers(cmd, ad, rd, work=work)
    assert np.array_equal(W.cpu().numpy().view(np.uint64), ref)
    # a second scan of changed costs reusing the grouping of the same allotment
    cm2 = (cm[:, ::-1] + 7).copy()
    ref2 = oracle.best_transfers(cm2, assign, rank.astype(np.int64))
    W2 = lb.best_transfers(torch.from_numpy(cm2).cuda(), ad, rd, work=work, reuse_grouping=True)
    assert np.array_equal(W2.cpu().numpy().view(np.uint64), ref2)


def test_full_scan_c3_size_bit_exact(lb):
    """The whole-matrix scan at the largest single-instance size (k=500,
    n=1,000,000, 2 GB of costs), on the processing order of that workload and
    its most-suitable-center allotment, against the oracle's definition."""
    import torch
    inst = L.make_config("C3")
    say("scan C3")
    smin, _, order, rank = oracle.setup(inst.cm)
    ref = oracle.best_transfers(inst.cm, smin, rank)
    W = lb.best_transfers(torch.from_numpy(inst.cm).cuda(), torch.from_numpy(smin).cuda(),
                          torch.from_numpy(rank.astype(np.int32)).cuda())
    assert np.array_equal(W.cpu().numpy().view(np.uint64), ref)


# ------------------------------------------ full-size properties (any size)
def test_c2_zero_capacity_closed_form(lb):
    """cap = 0 everywhere at the k=100, n=100,000 size: Equation (1) separates
    per unit, ASRAL reaches sum_d min_s CM(d,s) + pen[s] (closed form pinned
    against the exact optimum on small instances)."""
    import torch
    inst = L.make_config("C2")
    cap = np.zeros(inst.k, np.int32)
    say("C2 zero capacity")
    with lb.Instance(torch.from_numpy(inst.cm).cuda(), cap, inst.pen) as I:
        I.solve()
        obj, a = I.objective(), I.assignment()
    cmp = inst.cm.astype(np.int64) + inst.pen[None, :]
    assert obj == int(cmp.min(axis=1).sum())
    assert obj == pins.eq1(inst.cm, cap, inst.pen, a)


def test_c2_loose_capacity_is_row_argmin(lb):
    import torch
    inst = L.make_config("C2")
    cap = np.full(inst.k, inst.n, np.int32)
    say("C2 loose capacity")
    with lb.Instance(torch.from_numpy(inst.cm).cuda(), cap, inst.pen) as I:
        I.solve()
        obj, a = I.objective(), I.assignment()
    assert np.array_equal(a, np.argmin(inst.cm, axis=1))
    assert obj == int(inst.cm.min(axis=1).sum())


def test_c3_prefix_bit_exact_and_invariants(lb):
    """The k=500, n=1,000,000 workload: its first 2,000 iterations against the
    oracle (allotment, loads, objective, whole best-transfer table), then
    20,000 iterations checked through properties that hold at any size:
    Equation (1), no negative cycle (Lemmas 1-2), table = its definition."""
    import torch
    inst = L.make_config("C3")
    say("C3 prefix")
    _, _, order, rank = oracle.setup(inst.cm)
    with lb.Instance(torch.from_numpy(inst.cm).cuda(), inst.cap, inst.pen) as I:
        I.solve_iters(2000)
        ref = oracle.solve(*inst.arrays(), max_iters=2000, want_W=True)
        load, W, _ = I.snapshot()
        assert I.objective() == ref.objective
        assert np.array_equal(I.assignment(), ref.assign)
        assert np.array_equal(load, ref.load)
        assert np.array_equal(W, ref.W)
        I.solve_iters(18000)
        a = I.assignment()
        load, W, _ = I.snapshot()
        assert I.progress() == 20000
        assert I.objective() == pins.eq1(*inst.arrays(), a)
        assert np.array_equal(np.bincount(a[a >= 0], minlength=inst.k), load)
        assert np.array_equal(W, oracle.best_transfers(inst.cm, a, rank))
        assert not pins.has_negative_cycle(W)


# ---------------------------------------------------- options and autotuner
@pytest.mark.parametrize("k", [12, 40, 100, 131, 200, 300, 500])
def test_search_ratio_extremes_bit_exact(lb, k):
    """All Bellman-Ford rounds (ratio 0), Dijkstra order whenever the
    potentials allow it (ratio 2^20, bounded searches; with the table in
    global memory for k > 136) and the measured choice (-1) reach the
    oracle's allotment."""
    import torch
    inst = L.random_small(k=k, n=3000, seed=900 + k, cm_hi=400, pen_hi=300)
    say("search ratio", inst.name)
    ref = oracle.solve(*inst.arrays())
    for ratio in (0, 1 << 20, lb.SEARCH_AUTO):
        with lb.Instance(torch.from_numpy(inst.cm).cuda(), inst.cap, inst.pen) as I:
            I.set_option(lb.OPT_SEARCH_RATIO, ratio)
            assert I.get_option(lb.OPT_SEARCH_RATIO) == ratio
            I.solve()
            obj, a, st = I.objective(), I.assignment(), I.stats()
        say("  ratio", ratio, "dijkstra", st["dijkstra"], "bf_rounds", st["bf_rounds"])
        assert obj == ref.objective and np.array_equal(a, ref.assign)
        if ratio == 0:
            assert st["dijkstra"] == 0
        elif ratio == 1 << 20:
            assert st["dijkstra"] > 0 and st["dijkstra_settled"] >= st["dijkstra"]


@pytest.mark.parametrize("k", [12, 100, 200, 500])
def test_sink_potentials_bit_exact(lb, k):
    """Path searches on sink potentials (recomputed before every path search,
    or every fifth), in Dijkstra order and by the measured choice, reach the
    oracle's allotment."""
    import torch
    inst = L.random_small(k=k, n=3000, seed=700 + k, cm_hi=400, pen_hi=300)
    say("sink potentials", inst.name)
    ref = oracle.solve(*inst.arrays())
    for every, ratio in ((1, 1 << 20), (5, 1 << 20), (5, lb.SEARCH_AUTO)):
        with lb.Instance(torch.from_numpy(inst.cm).cuda(), inst.cap, inst.pen) as I:
            I.set_option(lb.OPT_SINK_EVERY, every)
            I.set_option(lb.OPT_SEARCH_RATIO, ratio)
            assert I.get_option(lb.OPT_SINK_EVERY) == every
            I.solve()
            obj, a, st = I.objective(), I.assignment(), I.stats()
        say("  every", every, "ratio", ratio, "sink", st["sink_potentials"], "settled", st["dijkstra_settled"])
        assert obj == ref.objective and np.array_equal(a, ref.assign)
        if st["path_searches"] > 0:
            assert st["sink_potentials"] > 0


def test_set_option_rejects_bad_values(lb):
    import torch
    inst = L.random_small(k=5, n=50, seed=3)
    with lb.Instance(torch.from_numpy(inst.cm).cuda(), inst.cap, inst.pen) as I:
        for opt, val in ((lb.OPT_SEARCH_RATIO, -2), (lb.OPT_SEARCH_RATIO, (1 << 20) + 1),
                         (lb.OPT_SINK_EVERY, -1), (lb.OPT_SINK_EVERY, (1 << 20) + 1), (99, 1)):
            with pytest.raises(lb.LbddError) as e:
                I.set_option(opt, val)
            assert e.value.code == lb.E_INVAL


def test_tune_search_records_ratio_and_stays_exact(lb):
    """The tuner times five search ratios on a prefix; the fastest becomes the
    default of new instances with that k, and the solve is unchanged."""
    import torch
    inst = L.random_small(k=29, n=6000, seed=29, cm_hi=500, pen_hi=400)
    say("tune search", inst.name)
    ratio, ms = lb.tune_search(torch.from_numpy(inst.cm).cuda(), inst.cap, inst.pen, iters=3000)
    say("  ratio", ratio, "ms", ms)
    assert len(ms) == len(lb.SEARCH_CANDIDATES) and all(t > 0 for t in ms)
    assert ratio in lb.SEARCH_CANDIDATES
    ref = oracle.solve(*inst.arrays())
    with lb.Instance(torch.from_numpy(inst.cm).cuda(), inst.cap, inst.pen) as I:
        assert I.get_option(lb.OPT_SEARCH_RATIO) == ratio
        I.solve()
        assert I.objective() == ref.objective and np.array_equal(I.assignment(), ref.assign)


@pytest.mark.parametrize("k,n", [(37, 20_000), (64, 50_000), (100, 100_000)])
def test_tune_best_transfers_bit_exact(lb, k, n):
    """Every tile configuration the tuner times gives the same table; the one
    it keeps is used by later scans of the same k."""
    import torch
    rng = np.random.default_rng(k + n)
    cm = rng.integers(0, 3000, size=(n, k), dtype=np.int64).astype(np.int32)
    assign = rng.integers(-1, k, size=n).astype(np.int32)
    rank = rng.permutation(n).astype(np.int32)
    say("tune scan", k, n)
    ref = oracle.best_transfers(cm, assign, rank.astype(np.int64))
    cmd, ad, rd = (torch.from_numpy(x).cuda() for x in (cm, assign, rank))
    W, cfg, ms, count = lb.tune_best_transfers(cmd, ad, rd, reps=2)
    say("  config", cfg, "ms", ms, "candidates", count)
    assert count >= 1
    vec, lpr, np_, waves = cfg
    assert vec in (1, 4) and lpr * np_ * vec >= k and waves in (1, 2)
    assert np.array_equal(W.cpu().numpy().view(np.uint64), ref)
    W2 = lb.best_transfers(cmd, ad, rd)
    assert np.array_equal(W2.cpu().numpy().view(np.uint64), ref)
