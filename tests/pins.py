"""Independent checks used to pin the oracle (and, on the GPU, the HIP path).

Nothing here calls the oracle or the HIP library: these are second
renderings of the paper's definitions or textbook/library results.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.optimize import linear_sum_assignment

KEY_NONE = np.uint64(0xFFFFFFFFFFFFFFFF)


def eq1(cm, cap, pen, assign) -> int:
    """Equation (1) with a constant per-unit penalty beyond capacity."""
    cm = np.asarray(cm, np.int64)
    a = np.asarray(assign)
    ok = a >= 0
    total = int(cm[np.nonzero(ok)[0], a[ok]].sum())
    load = np.bincount(a[ok], minlength=cm.shape[1])
    over = np.maximum(0, load - np.asarray(cap, np.int64))
    return total + int((over * np.asarray(pen, np.int64)).sum())


def table_penalty(off, val, s: int, j: int) -> int:
    """Penalty of the j-th unit (j >= 1) beyond the capacity of center s: the
    j-th value of the center's table, its last value for every later unit."""
    lo, hi = int(off[s]), int(off[s + 1])
    return int(val[lo + min(j, hi - lo) - 1])


def eq2(cm, cap, off, val, assign) -> int:
    """Equation (2): the sum of CM over the allotment plus, for every center,
    the penalties of its 1st .. (load - capacity)-th units beyond capacity."""
    cm = np.asarray(cm, np.int64)
    a = np.asarray(assign)
    ok = a >= 0
    total = int(cm[np.nonzero(ok)[0], a[ok]].sum())
    load = np.bincount(a[ok], minlength=cm.shape[1])
    for s in range(cm.shape[1]):
        for j in range(1, int(load[s]) - int(cap[s]) + 1):
            total += table_penalty(off, val, s, j)
    return total


def opt_convex(cm, cap, off, val) -> int:
    """Exact optimum of Equation (2) for non-decreasing penalties: center s
    offers cap[s] slots at CM(d,s) and then, for j = 1..n, a slot at CM(d,s)
    plus the j-th overload penalty.  The penalties do not decrease, so an
    optimal matching fills each center's slots in order and its cost is the
    objective; scipy's assignment solver finds it."""
    cm = np.asarray(cm, np.int64)
    n, k = cm.shape
    cols = []
    for s in range(k):
        cols += [cm[:, s]] * int(min(cap[s], n))
        cols += [cm[:, s] + table_penalty(off, val, s, j) for j in range(1, n + 1)]
    cost = np.stack(cols, axis=1)
    r, c = linear_sum_assignment(cost)
    return int(cost[r, c].sum())


def opt_brute(cm, cap, pen) -> int:
    """Exact optimum of Equation (1) by enumerating all k^n complete allotments."""
    cm = np.asarray(cm, np.int64)
    n, k = cm.shape
    best = None
    for a in itertools.product(range(k), repeat=n):
        v = eq1(cm, cap, pen, np.array(a))
        best = v if best is None or v < best else best
    return best


def opt_assignment(cm, cap, pen) -> int:
    """Exact optimum via min-cost bipartite matching with center copies (the
    reduction the paper compares against, Introduction and Section 5): center
    s gets n slots, the first cap[s] at cost CM(d,s), the rest at
    CM(d,s) + pen[s]; scipy's Hungarian-type solver matches units to slots."""
    cm = np.asarray(cm, np.int64)
    n, k = cm.shape
    cols = []
    for s in range(k):
        extra = np.where(np.arange(n) >= cap[s], int(pen[s]), 0)
        cols.append(cm[:, s:s + 1] + extra[None, :])
    cost = np.concatenate(cols, axis=1)
    r, c = linear_sum_assignment(cost)
    return int(cost[r, c].sum())


def key_delta(W):
    return (np.asarray(W, np.uint64) >> np.uint64(32)).astype(np.int64) - 2**31


def has_negative_cycle(W) -> bool:
    """Floyd-Warshall on the condensed Gamma graph (edge u->v = delta of W[u][v])."""
    W = np.asarray(W, np.uint64)
    k = W.shape[0]
    INF = np.int64(2**62)
    D = np.where(W == KEY_NONE, INF, key_delta(W)).astype(np.int64)
    np.fill_diagonal(D, np.minimum(np.diag(D), 0))
    for m in range(k):
        D = np.minimum(D, np.where((D[:, m:m + 1] < INF) & (D[m:m + 1, :] < INF),
                                   D[:, m:m + 1] + D[m:m + 1, :], INF))
    return bool((np.diag(D) < 0).any())


def split_graph(W, anchor, mode, load, cap, pen):
    """Edge dict {(u,v): cost} of NCyc (mode 0) or NPath (mode 1), nodes
    0..k-1 with the anchor as s*_out and node k as s*_in (Sections 3.3-3.4)."""
    W = np.asarray(W, np.uint64)
    k = W.shape[0]
    dl = key_delta(W)
    E = {}
    for u in range(k):
        for v in range(k):
            if u != v and v != anchor and W[u, v] != KEY_NONE:
                E[(u, v)] = int(dl[u, v])
    for u in range(k):
        if u == anchor:
            continue
        if mode == 0:
            if W[u, anchor] != KEY_NONE:
                E[(u, k)] = int(dl[u, anchor])
        else:
            q = int(pen[u]) if load[u] >= cap[u] else 0
            E[(u, k)] = q - int(pen[anchor])
    return E


def min_simple_path(E, k, src):
    """Minimum cost over all simple src -> k paths, by enumeration (None if no path)."""
    others = [v for v in range(k) if v != src]
    best = None
    for L in range(0, len(others) + 1):
        for mid in itertools.permutations(others, L):
            nodes = (src, *mid, k)
            cost = 0
            ok = True
            for a, b in zip(nodes, nodes[1:]):
                if (a, b) not in E:
                    ok = False
                    break
                cost += E[(a, b)]
            if ok and (best is None or cost < best):
                best = cost
    return best


def opt_strict(cm, cap) -> int:
    """Exact optimum of strict-LBDD (Appendix B, Equation (3)): center s gets
    cap[s] slots at cost CM(d,s); with excess demand n - sum(cap) more slots
    at a cost above every CM entry take the units no center can hold (their
    cost, the same for every complete allotment, is subtracted); scipy's
    assignment solver matches units to slots."""
    cm = np.asarray(cm, np.int64)
    n, k = cm.shape
    total = int(np.sum(cap))
    big = int(cm.max()) + 1
    cols = [np.repeat(cm[:, s:s + 1], int(cap[s]), axis=1) for s in range(k) if cap[s] > 0]
    excess = max(0, n - total)
    if excess:
        cols.append(np.full((n, excess), big, np.int64))
    cost = np.concatenate(cols, axis=1)
    r, c = linear_sum_assignment(cost)
    return int(cost[r, c].sum()) - excess * big


def strict_brute(cm, cap) -> int:
    """Strict-LBDD optimum by enumerating every allotment that respects the
    capacities (units beyond the total capacity may stay unallotted, exactly
    max(0, n - sum(cap)) of them, at no cost)."""
    cm = np.asarray(cm, np.int64)
    n, k = cm.shape
    excess = max(0, n - int(np.sum(cap)))
    best = None
    for a in itertools.product(range(-1, k), repeat=n):
        a = np.array(a)
        if int((a < 0).sum()) != excess:
            continue
        if any(int((a == s).sum()) > cap[s] for s in range(k)):
            continue
        v = int(sum(cm[d, a[d]] for d in range(n) if a[d] >= 0))
        best = v if best is None or v < best else best
    return best
