"""CPU model of the refill merge's lane operations (solve.hip, refill_column).

A refill puts the BEST_M smallest keys of a center's member rows into a
best-transfer list (definition of Gamma).  Each wavefront takes its BEST_M
smallest by BEST_M wavefront minima, and wavefront 0 merges the 16 * BEST_M
candidates.  The wavefront minimum (wave_min_u32 / wave_min_u64) is modelled
here lane by lane: DPP moves within rows of 16 lanes (quad permutations, half
row mirror, row mirror) with bound_ctrl set, then the 16- and 32-lane row
swaps, high words before low words.  The model also says what a lane that
is switched off in the exec mask contributes: a DPP read of a disabled lane
with bound_ctrl set yields 0, so a minimum taken with some lanes off can come
out as 0, which as a list key is the most negative delta there is."""
import numpy as np
import pytest

BEST_M = 8
NT = 1024
KEY_NONE = (1 << 64) - 1
U32 = 0xFFFFFFFF


def _dpp(x, exec_, src_of_lane):
    """mov_dpp with row and bank masks all set and bound_ctrl set: every
    active lane reads its source lane, or 0 where that lane is disabled."""
    out = x.copy()
    for lane in range(64):
        if exec_[lane]:
            src = src_of_lane(lane)
            out[lane] = x[src] if exec_[src] else 0
    return out


def _swap(x, rows):
    """permlane16/32 swap of a register with itself: the two results, per
    lane its own row's value and its partner row's (order per the swap)."""
    a = x.copy()
    b = x.copy()
    n = 64 // rows
    for blk in range(0, 64, 2 * n):
        lo = slice(blk, blk + n)
        hi = slice(blk + n, blk + 2 * n)
        a[hi] = x[lo]      # odd part of the first operand takes the even part of the second
        b[lo] = x[hi]
    return a, b


def wave_min_u32(x, exec_):
    x = np.asarray(x, dtype=np.uint64) & U32
    steps = [lambda l: (l & ~3) + [1, 0, 3, 2][l & 3],
             lambda l: (l & ~3) + [2, 3, 0, 1][l & 3],
             lambda l: (l & ~7) + (7 - (l & 7)),
             lambda l: (l & ~15) + (15 - (l & 15))]
    for f in steps:
        y = _dpp(x, exec_, f)
        x = np.where(exec_, np.minimum(x, y), x)
    for rows in (4, 2):
        a, b = _swap(x, rows)
        x = np.where(exec_, np.minimum(x, np.minimum(a, b)), x)
    return x


def _first_active(x, exec_):
    return int(x[int(np.argmax(exec_))])


def wave_min_u64(x, exec_):
    x = [int(v) for v in x]
    hi = _first_active(wave_min_u32([v >> 32 for v in x], exec_), exec_)
    lo_in = [(v & U32) if (v >> 32) == hi else U32 for v in x]
    lo = _first_active(wave_min_u32(lo_in, exec_), exec_)
    return (hi << 32) | lo


def _merge(lst, q):
    """list_merge: q enters the sorted list, the largest falls off."""
    return sorted(lst + [q])[:BEST_M]


def refill_model(keys, exec0=None):
    """The kernel's refill of one list from member keys (member i read by
    thread i mod NT).  exec0: the exec mask wavefront 0 runs its merge with
    (all lanes in the kernel)."""
    lists = [[KEY_NONE] * BEST_M for _ in range(NT)]
    for i, q in enumerate(keys):
        lists[i % NT] = _merge(lists[i % NT], q)
    full = np.ones(64, bool)
    cand = []
    for w in range(NT // 64):
        b = [list(lists[w * 64 + l]) for l in range(64)]
        for _ in range(BEST_M):
            g = wave_min_u64([bl[0] for bl in b], full)
            cand.append(g)
            if g != KEY_NONE:
                owners = [l for l in range(64) if b[l][0] == g]
                assert len(owners) == 1
                b[owners[0]] = b[owners[0]][1:] + [KEY_NONE]
    assert len(cand) == 128
    ex = full if exec0 is None else exec0
    c0 = [min(cand[l], cand[l + 64]) for l in range(64)]
    c1 = [max(cand[l], cand[l + 64]) for l in range(64)]
    out = []
    for _ in range(BEST_M):
        g = wave_min_u64(c0, ex)
        out.append(g)
        if g != KEY_NONE:
            for l in range(64):
                if c0[l] == g:
                    c0[l], c1[l] = c1[l], KEY_NONE
                    break
    return out


def _keys(rng, m):
    """Unique packed keys ((delta + 2^31) << 32) | rank, ranks distinct."""
    deltas = rng.integers(-3000, 3000, size=m)
    ranks = rng.permutation(10 * m + 10)[:m]
    return [((int(d) + (1 << 31)) << 32) | int(r) for d, r in zip(deltas, ranks)]


def test_wave_minimum_with_every_lane_active():
    rng = np.random.default_rng(1)
    full = np.ones(64, bool)
    for _ in range(200):
        x = [int(v) for v in rng.integers(0, 1 << 63, size=64, dtype=np.uint64)]
        if rng.random() < 0.3:
            x[int(rng.integers(64))] = KEY_NONE
        assert wave_min_u64(x, full) == min(x)
        v = rng.integers(0, 1 << 32, size=64, dtype=np.uint64)
        assert int(wave_min_u32(v, full)[int(rng.integers(64))]) == int(v.min())


@pytest.mark.parametrize("m", [0, 1, 5, 8, 9, 64, 200, 1556, 3000])
def test_refill_merge_gives_the_smallest_keys(m):
    rng = np.random.default_rng(m)
    keys = _keys(rng, m)
    want = sorted(keys)[:BEST_M] + [KEY_NONE] * max(0, BEST_M - m)
    assert refill_model(keys) == want


def test_refill_merge_with_lanes_switched_off_yields_key_zero():
    """The failure mode of a minimum taken with lanes off: a DPP read of a
    disabled lane gives 0, so the head of the refilled list becomes key 0,
    delta -2^31, an edge no cycle can balance (every other delta is above
    -2^31 and below 2^31): Bellman-Ford then reports a negative cycle, the
    status the withdrawn per-wavefront merge stopped with."""
    rng = np.random.default_rng(7)
    keys = _keys(rng, 500)
    exec0 = np.ones(64, bool)
    exec0[20:] = False                      # e.g. a merge run by lanes < 20 only: row 1
                                            # reads its disabled lanes 20..31 as 0
    out = refill_model(keys, exec0)
    assert out[0] == 0
    # a whole row of lanes switched off is read only through the row swaps,
    # which move the disabled lanes' registers as they are: no zero then
    exec1 = np.ones(64, bool)
    exec1[16:] = False
    assert refill_model(keys, exec1)[0] != 0
    delta = (out[0] >> 32) - (1 << 31)
    assert delta == -(1 << 31)
    # any back edge of |delta| < 2^31 closes a negative two-center cycle
    assert delta + ((1 << 31) - 1) < 0
