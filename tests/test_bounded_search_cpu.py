"""The solve kernel's bounded search in Dijkstra order, modelled on the CPU and
checked against the oracle's synchronous Bellman-Ford rounds.

With node potentials pot that are feasible (w(u, v) + pot[u] - pot[v] >= 0)
on every edge except those leaving the anchor s, the kernel settles centers in
the order of (reduced label, edges), but only while a settled center can still
matter for s_in:
  * cycle mode (NCyc, Algorithm 1): an edge u -> s is feasible, so the cycle
    through u costs at least u's reduced label; after s itself, centers are
    settled while the smallest open reduced label is negative;
  * path mode (NPath, Appendix A; every edge feasible): u's penalty edge gives
    s_in at least (u's reduced label) + Pmin, Pmin the smallest
    pot[u] + w(u, s_in) - pot[s]; centers are settled until that bound
    exceeds both -1 and the best s_in candidate found so far.
s_in then follows from the settled labels by the same rule as after full
rounds (smallest candidate, then the earliest hop, then the smallest center).
The claims checked here:
  1. the s_in label and the whole predecessor chain equal the oracle's
     whenever the oracle's s_in label is negative (a refinement applies), and
     the bounded search finds no negative label when the oracle finds none;
  2. the new potentials (settled: the label; open: pot - pot[s] + D, D the
     reduced label the search stopped at, at least 0) are feasible on every
     edge when nothing applies, and on every edge outside row s and column s
     when something does (those are checked on the device after the moves).
The model breaks ties between equal keys at random."""
import numpy as np
import pytest

import oracle
from tests import pins


def _delta(key):
    return int(key >> np.uint64(32)) - 2**31


def _key(d, rank):
    return np.uint64(((int(d) + 2**31) << 32) | int(rank))


def _case(seed, mode):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 12))
    pot = rng.integers(-8, 9, size=k)
    s = int(rng.integers(0, k))
    W = np.full((k, k), pins.KEY_NONE, np.uint64)
    for u in range(k):
        for v in range(k):
            # the anchor holds a unit, so it has an edge to every center
            if u != v and (u == s or rng.random() < 0.7):
                W[u, v] = _key(pot[v] - pot[u] + rng.integers(0, 3), rng.integers(0, 99))
    if mode == 0:
        # the unit that just joined the anchor may lower its row anywhere
        for v in range(k):
            if v != s and rng.random() < 0.5:
                W[s, v] = _key(_delta(W[s, v]) - int(rng.integers(0, 9)), rng.integers(0, 99))
        load = np.zeros(k, np.int32)
        cap = np.zeros(k, np.int32)
        pen = np.ones(k, np.int32)
    else:
        load = rng.integers(0, 6, size=k).astype(np.int32)
        cap = rng.integers(0, 6, size=k).astype(np.int32)
        cap[s] = max(0, int(load[s]) - 1)          # the anchor is overloaded
        load[s] = max(int(load[s]), int(cap[s]) + 1)
        pen = rng.integers(1, 25, size=k).astype(np.int32)
    return rng, k, pot, W, s, load, cap, pen


def bounded_search(W, s, pot, mode, load, cap, pen, rng):
    """Returns (dist_sin, pred of every settled node incl. s_in, labels, new
    potentials, settled count)."""
    k = W.shape[0]

    def in_weight(u):
        if u == s:
            return None
        if mode == 0:
            return None if W[u, s] == pins.KEY_NONE else _delta(W[u, s])
        return (int(pen[u]) if load[u] >= cap[u] else 0) - int(pen[s])

    pmin = None
    if mode == 1:
        pmin = min(int(pot[u]) + in_weight(u) - int(pot[s]) for u in range(k) if u != s)
    lab = {s: (0, 0, -1)}                        # (distance, edges, predecessor)
    settled = []
    best = None
    D = None
    while True:
        open_ = [v for v in lab if v not in settled]
        if not open_:
            top = max(lab[v][0] - int(pot[v]) + int(pot[s]) for v in settled)
            D = max(top, 0)
            break
        key = {v: (lab[v][0] - int(pot[v]) + int(pot[s]), lab[v][1]) for v in open_}
        m = min(key.values())
        if settled and mode == 0 and m[0] >= 0:
            D = m[0]
            break
        if settled and mode == 1 and m[0] + pmin > min(-1 if best is None else best, -1):
            D = m[0]
            break
        ties = [v for v in open_ if key[v] == m]
        u = ties[int(rng.integers(0, len(ties)))]
        settled.append(u)
        if mode == 1 and u != s:
            c = lab[u][0] + in_weight(u)
            best = c if best is None else min(best, c)
        for v in range(k):
            if v == s or v in settled or W[u, v] == pins.KEY_NONE:
                continue
            cand = (lab[u][0] + _delta(W[u, v]), lab[u][1] + 1, u)
            if v not in lab or cand < lab[v]:
                lab[v] = cand
    # s_in from the settled labels: smallest candidate, earliest hop, smallest u
    cands = [(lab[u][0] + in_weight(u), lab[u][1], u) for u in settled
             if u != s and in_weight(u) is not None]
    dist_sin, pred_sin = None, -1
    if cands:
        c = min(cands)
        dist_sin, pred_sin = c[0], c[2]
    pred = {v: lab[v][2] for v in settled}
    pred[k] = pred_sin
    newpot = [lab[v][0] if v in settled else int(pot[v]) - int(pot[s]) + D for v in range(k)]
    return dist_sin, pred, {v: lab[v][0] for v in settled}, newpot, len(settled)


def _feasible(W, p, skip_s=None):
    k = W.shape[0]
    for u in range(k):
        for v in range(k):
            if u == v or W[u, v] == pins.KEY_NONE:
                continue
            if skip_s is not None and (u == skip_s or v == skip_s):
                continue
            if p[v] > p[u] + _delta(W[u, v]):
                return False
    return True


def _chain(pred, k, s):
    out, v = [], k
    while v != -1 and len(out) <= k + 1:
        out.append(int(v))
        if v == s:
            break
        v = pred[v]
    return out


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("seed", range(150))
def test_bounded_search_matches_synchronous_rounds(seed, mode):
    rng, k, pot, W, s, load, cap, pen = _case(seed, mode)
    dist, pred, _ = oracle.refine_search(W, s, mode, load, cap, pen)
    D_ref = int(dist[k]) if dist[k] != oracle.DIST_NONE else None
    for _ in range(4):
        d, bpred, labels, newpot, nset = bounded_search(W, s, pot, mode, load, cap, pen, rng)
        # every settled label is the shortest distance
        for v, x in labels.items():
            if v != s:
                assert x == dist[v], (seed, mode, v)
        if D_ref is not None and D_ref < 0:
            assert d == D_ref, (seed, mode)
            assert _chain(bpred, k, s) == _chain({**{v: int(pred[v]) for v in range(k + 1)}}, k, s)
            # only row s and column s may be infeasible (checked after the moves)
            assert _feasible(W, newpot, skip_s=s), (seed, mode)
        else:
            assert d is None or d >= 0, (seed, mode, d, D_ref)
            assert _feasible(W, newpot), (seed, mode)
        assert newpot[s] == 0


def test_bounded_search_settles_few_centers_when_the_drop_is_small():
    """The point of the bound: a small drop in the anchor's row settles a
    handful of centers, not all of them."""
    rng = np.random.default_rng(7)
    k = 60
    pot = rng.integers(-50, 51, size=k)
    W = np.full((k, k), pins.KEY_NONE, np.uint64)
    for u in range(k):
        for v in range(k):
            if u != v:
                W[u, v] = _key(pot[v] - pot[u] + rng.integers(5, 40), u)
    s = 3
    W[s, 10] = _key(pot[10] - pot[s] - 2, 0)     # reduced weight -2
    z = np.zeros(k, np.int32)
    _, _, _, _, nset = bounded_search(W, s, pot, 0, z, z, np.ones(k, np.int32), rng)
    assert nset <= 3


def pruned_rounds(W, s, pot, mode, load, cap, pen):
    """The kernel's pruned Bellman-Ford rounds: synchronous rounds from s in
    which a center whose label dropped enters the next frontier only while
    its reduced label r = dist + pot[s] - pot[v] is below Db (cycle mode 0,
    path mode -Pmin).  Returns (dist_sin, pred, labels of the centers below
    Db, new potentials)."""
    k = W.shape[0]

    def in_weight(u):
        if u == s:
            return None
        if mode == 0:
            return None if W[u, s] == pins.KEY_NONE else _delta(W[u, s])
        return (int(pen[u]) if load[u] >= cap[u] else 0) - int(pen[s])

    if mode == 0:
        Db = 0
    else:
        others = [int(pot[u]) + in_weight(u) - int(pot[s]) for u in range(k) if u != s]
        Db = -min(others) if others else -(1 << 46)
    INF = (float("inf"), 0, 0)
    lab = [INF] * k
    lab[s] = (0, 0, -1)
    front = [s]
    for _ in range(k + 1):
        new = list(lab)
        for v in range(k):
            if v == s:
                continue
            for u in front:
                if W[u, v] == pins.KEY_NONE:
                    continue
                c = (lab[u][0] + _delta(W[u, v]), lab[u][1] + 1, u)
                if c < new[v]:
                    new[v] = c
        nxt = [v for v in range(k) if new[v] < lab[v]
               and new[v][0] + int(pot[s]) - int(pot[v]) < Db]
        lab = new
        if not nxt:
            break
        front = nxt
    rel = [v for v in range(k) if lab[v] is not INF and
           (v == s or lab[v][0] + int(pot[s]) - int(pot[v]) < Db)]
    cands = [(lab[u][0] + in_weight(u), lab[u][1], u) for u in rel if u != s and in_weight(u) is not None]
    dist_sin, pred_sin = (None, -1)
    if cands:
        c = min(cands)
        dist_sin, pred_sin = c[0], c[2]
    pred = {v: lab[v][2] for v in rel}
    pred[k] = pred_sin
    D = max(Db, 0)
    newpot = [lab[v][0] if v in rel else int(pot[v]) - int(pot[s]) + D for v in range(k)]
    return dist_sin, pred, {v: lab[v][0] for v in rel}, newpot


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("seed", range(150))
def test_pruned_rounds_match_synchronous_rounds(seed, mode):
    """Pruned Bellman-Ford (the kernel's rounds while potentials are feasible)
    gives the oracle's s_in label and path whenever a refinement applies, no
    negative label otherwise, exact labels below the bound, and potentials
    feasible where the bounded Dijkstra search's are."""
    _, k, pot, W, s, load, cap, pen = _case(seed, mode)
    dist, pred, _ = oracle.refine_search(W, s, mode, load, cap, pen)
    D_ref = int(dist[k]) if dist[k] != oracle.DIST_NONE else None
    d, bpred, labels, newpot = pruned_rounds(W, s, pot, mode, load, cap, pen)
    for v, x in labels.items():
        if v != s:
            assert x == dist[v], (seed, mode, v)
    if D_ref is not None and D_ref < 0:
        assert d == D_ref, (seed, mode)
        assert _chain(bpred, k, s) == _chain({v: int(pred[v]) for v in range(k + 1)}, k, s)
        assert _feasible(W, newpot, skip_s=s), (seed, mode)
    else:
        assert d is None or d >= 0, (seed, mode, d, D_ref)
        assert _feasible(W, newpot), (seed, mode)
    assert newpot[s] == 0


def windowed_rounds(W, s, pot, mode, load, cap, pen, width, counts=None):
    """The kernel's windowed rounds: centers whose label dropped are pending,
    ordered by their window key (reduced distance, then edges).  s goes
    first, alone; then each window starts at the smallest pending key lo and
    relaxes, round after round, the pending centers with keys below
    lo + width (width in key units: one unit of reduced distance is 2^11).
    A dropped label makes its center pending only below Db.  Returns the
    labels, from which the result follows as for pruned rounds; counts, when
    given, receives how often each center was relaxed."""
    k = W.shape[0]

    def in_weight(u):
        if mode == 0:
            return None if W[u, s] == pins.KEY_NONE else _delta(W[u, s])
        return (int(pen[u]) if load[u] >= cap[u] else 0) - int(pen[s])

    if mode == 0:
        Db = 0
    else:
        others = [int(pot[u]) + in_weight(u) - int(pot[s]) for u in range(k) if u != s]
        Db = -min(others) if others else -(1 << 46)
    INF = (float("inf"), 0, 0)
    lab = [INF] * k
    lab[s] = (0, 0, -1)
    pend = {s}
    r = lambda v: lab[v][0] + int(pot[s]) - int(pot[v])
    key = lambda v: (r(v) << 11) | lab[v][1]

    def relax(front):
        new = list(lab)
        for v in range(k):
            if v == s:
                continue
            for u in front:
                if W[u, v] == pins.KEY_NONE:
                    continue
                c = (lab[u][0] + _delta(W[u, v]), lab[u][1] + 1, u)
                if c < new[v]:
                    new[v] = c
        for u in front:
            if counts is not None:
                counts[u] += 1
        return new

    pend.discard(s)
    lab = relax([s])
    pend |= {v for v in range(k) if lab[v] is not INF and v != s and r(v) < Db}
    while pend:
        lo = min(key(v) for v in pend)
        if lo >= Db << 11:
            break
        while True:
            front = sorted(v for v in pend if key(v) < lo + width)
            if not front:
                break
            pend -= set(front)
            new = relax(front)
            for v in range(k):
                if new[v] < lab[v] and new[v][0] + int(pot[s]) - int(pot[v]) < Db:
                    pend.add(v)
            lab = new
    rel = [v for v in range(k) if lab[v] is not INF and (v == s or r(v) < Db)]
    return {v: lab[v] for v in rel}


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("seed", range(100))
def test_windowed_rounds_give_the_pruned_labels(seed, mode):
    """Windowed rounds (any window width) give every center below the bound
    the labels of the synchronous rounds, predecessor included, so the s_in
    result and the potentials are those of pruned rounds."""
    rng, k, pot, W, s, load, cap, pen = _case(seed, mode)
    dist, pred, _ = oracle.refine_search(W, s, mode, load, cap, pen)
    _, _, labels_p, _ = pruned_rounds(W, s, pot, mode, load, cap, pen)
    for width in (1, 3, 2 ** 11, 3 * 2 ** 11 + 5, 10 ** 12):
        labs = windowed_rounds(W, s, pot, mode, load, cap, pen, width)
        assert set(labs) == set(labels_p), (seed, mode, width)
        for v, (d, e, p) in labs.items():
            if v != s:
                assert d == dist[v] and p == pred[v], (seed, mode, width, v)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("seed", range(60))
def test_width_one_windows_relax_each_center_once(seed, mode):
    """With width 1 a window holds one key, and the pending center with the
    smallest key is final, so no center is relaxed twice."""
    rng, k, pot, W, s, load, cap, pen = _case(seed, mode)
    counts = [0] * k
    windowed_rounds(W, s, pot, mode, load, cap, pen, 1, counts)
    assert max(counts) <= 1, (seed, mode, counts)


def test_one_wide_window_relaxes_centers_again():
    """The contrast: one window over every key relaxes a center whose label
    drops again (most of these inputs have one)."""
    again = 0
    for mode in (0, 1):
        for seed in range(60):
            rng, k, pot, W, s, load, cap, pen = _case(seed, mode)
            counts = [0] * k
            windowed_rounds(W, s, pot, mode, load, cap, pen, 10 ** 12, counts)
            again += max(counts) > 1
    assert again > 30


def windowed_threads(W, s, pot, mode, load, cap, pen, width, T, G, rng):
    """The kernel's windowed loop at the level of its threads: T threads for
    the pass over the pending flags, G threads per target for the
    relaxations (frontier entries g, g + G, ...), the counters of a round in
    one of three rotating slots (slot c + 1 cleared by thread 0 at the start
    of round c), labels packed as the kernel packs them, and between two
    barriers every thread's steps interleaved at random.  Each thread takes
    the window decision of a round after that round's second barrier, while
    faster threads already run the next round's pass (no barrier between
    them).  Returns the labels below the bound; asserts that every thread
    takes the same decisions."""
    k = W.shape[0]

    def in_weight(u):
        if mode == 0:
            return None if W[u, s] == pins.KEY_NONE else _delta(W[u, s])
        return (int(pen[u]) if load[u] >= cap[u] else 0) - int(pen[s])

    if mode == 0:
        Db = 0
    else:
        others = [int(pot[u]) + in_weight(u) - int(pot[s]) for u in range(k) if u != s]
        Db = -min(others) if others else -(1 << 46)
    NONE = (1 << 64) - 1
    LB = 1 << 41
    pack = lambda d, e, p: ((d + LB) << 22) | (e << 11) | p
    dist = lambda l: (l >> 22) - LB
    lab = [NONE] * k
    lab[s] = pack(0, 0, 0)
    pend = [v == s for v in range(k)]
    r = lambda l, v: dist(l) + int(pot[s]) - int(pot[v])
    wkey = lambda l, v: ((r(l, v) + (1 << 46)) << 11) | ((l >> 11) & 0x7FF)
    key_db = (Db + (1 << 46)) << 11
    nfront = [0, 0, 0]
    wlo = [NONE, NONE, NONE]
    front = []                                  # (center, base) taken in the round
    hi0 = wkey(lab[s], s) + 1
    st = [dict(hi=hi0, win=0, done=False) for _ in range(T)]
    log = [[] for _ in range(T)]                # each thread's decisions

    def run_interleaved(progs):
        live = list(progs)
        while live:
            i = int(rng.integers(len(live)))
            try:
                next(live[i])
            except StopIteration:
                live.pop(i)

    prev = None                                 # slot of the round whose decision is pending
    for it in range(4 * k + 16):
        c = it % 3

        def step(t):
            h = st[t]
            if prev is not None:                # the previous round's window decision
                lo = wlo[prev]
                yield
                if lo >= h["hi"] or h["win"] == 0:
                    if lo == NONE or lo >= key_db:
                        h["done"] = True
                    else:
                        h["hi"] = lo + width
                        h["win"] += 1
                log[t].append((h["hi"], h["win"], h["done"]))
                if h["done"]:
                    return
            if t == 0:
                nfront[(c + 1) % 3] = 0
                wlo[(c + 1) % 3] = NONE
                yield
            for v in range(t, k, T):
                if pend[v]:
                    l = lab[v]
                    key = wkey(l, v)
                    yield
                    if key < h["hi"]:
                        pend[v] = False
                        front.append((v, (l & ~0x7FF) + (1 << 11) + v))
                        nfront[c] += 1
                    else:
                        wlo[c] = min(wlo[c], key)
                    yield
        run_interleaved([step(t) for t in range(T)])
        assert all(x == log[0] for x in log)
        if st[0]["done"]:
            break
        nf = nfront[c]                          # barrier: every thread reads it
        if nf == 0:
            break
        assert nf == len(front)
        entries = list(front)
        front.clear()

        def relax(v, g):
            best = NONE
            for (u, base) in entries[g::G]:
                if W[u, v] != pins.KEY_NONE:
                    best = min(best, base + (_delta(W[u, v]) << 22))
                yield
            old = lab[v]                        # atomic minimum, old value returned
            lab[v] = min(old, best)
            if best < old and r(best, v) < Db:
                pend[v] = True
                wlo[c] = min(wlo[c], wkey(best, v))
            yield
        run_interleaved([relax(v, g) for v in range(k) if v != s for g in range(G)])
        prev = c                                # barrier; the decision runs in the next pass
    rel = [v for v in range(k) if lab[v] != NONE and (v == s or r(lab[v], v) < Db)]
    return {v: (dist(lab[v]), (lab[v] >> 11) & 0x7FF, (lab[v] & 0x7FF) if v != s else -1) for v in rel}


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("seed", range(40))
def test_windowed_threads_match_the_pruned_labels(seed, mode):
    """The windowed loop as its threads run it (rotating counter slots,
    interleaved steps, one barrier between a round's pass and its
    relaxations and one after) reaches the labels of pruned rounds, and every
    thread takes the same window decisions."""
    rng, k, pot, W, s, load, cap, pen = _case(seed, mode)
    dist, pred, _ = oracle.refine_search(W, s, mode, load, cap, pen)
    _, _, labels_p, _ = pruned_rounds(W, s, pot, mode, load, cap, pen)
    for width in (1, 2 ** 11, 10 ** 12):
        for T, G in ((1, 1), (3, 2), (8, 3)):
            labs = windowed_threads(W, s, pot, mode, load, cap, pen, width, T, G, rng)
            assert set(labs) == set(labels_p), (seed, mode, width, T)
            for v, (d, e, p) in labs.items():
                if v != s:
                    assert d == dist[v] and p == pred[v], (seed, mode, width, T, v)
