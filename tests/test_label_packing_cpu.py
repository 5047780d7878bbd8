"""The search labels' bit budget, checked on the CPU with 64-bit wraparound
arithmetic.

The solve kernel packs a center's label as ((dist + 2^41) << 22) |
(edges << 11) | pred, so one unsigned 64-bit minimum orders by (distance,
edges, predecessor), and it relaxes an edge with delta (the key's high word
minus 2^31) as (label & ~0x7ff) + (delta << 22) + (1 << 11) + u.  A simple
path has at most k - 1 <= 2047 edges of |delta| < 2^30, so its distance lies
within +-2^41 and all three fields fit.  These tests check the order and the
relaxation at the extremes of those ranges."""
import numpy as np
import pytest

MASK = 2**64 - 1
BIAS = 2**41
MAX_K = 2048
DMAX = (MAX_K - 1) * (2**30 - 1)                 # the longest simple path's |distance|


def pack(dist, edges, pred):
    return (((dist + BIAS) << 22) | (edges << 11) | pred) & MASK


def relax(label, delta, u):
    """The kernel's candidate through an edge out of u (uint64 wraparound)."""
    return ((label & ~0x7ff & MASK) + ((delta << 22) & MASK) + (1 << 11) + u) & MASK


def unpack(x):
    return (x >> 22) - BIAS, (x >> 11) & 0x7ff, x & 0x7ff


def _labels(rng, m):
    d = rng.integers(-DMAX, DMAX + 1, size=m)
    e = rng.integers(0, MAX_K, size=m)
    p = rng.integers(0, MAX_K, size=m)
    ext = [(-DMAX, 0, 0), (DMAX, MAX_K - 1, MAX_K - 1), (0, 0, 0), (-DMAX, MAX_K - 1, 0),
           (DMAX, 0, MAX_K - 1)]
    return [(int(a), int(b), int(c)) for a, b, c in zip(d, e, p)] + ext


@pytest.mark.parametrize("seed", range(5))
def test_packed_order_is_the_lexicographic_order(seed):
    rng = np.random.default_rng(seed)
    labs = _labels(rng, 400)
    # ties in distance and edges are common in the searches: make some
    labs += [(labs[i][0], labs[i][1], int(rng.integers(0, MAX_K))) for i in range(50)]
    labs += [(labs[i][0], int(rng.integers(0, MAX_K)), labs[i][2]) for i in range(50)]
    by_tuple = sorted(labs)
    by_packed = sorted(labs, key=lambda t: pack(*t))
    assert by_tuple == by_packed
    for t in labs:
        assert 0 <= pack(*t) < 2**64 and unpack(pack(*t)) == t


@pytest.mark.parametrize("seed", range(5))
def test_relaxation_is_the_packed_extension(seed):
    rng = np.random.default_rng(100 + seed)
    for _ in range(2000):
        edges = int(rng.integers(0, MAX_K - 1))          # a simple path one edge short
        delta = int(rng.integers(-(2**30) + 1, 2**30))
        lo = max(-DMAX, -DMAX - delta)
        hi = min(DMAX, DMAX - delta)
        dist = int(rng.integers(lo, hi + 1))
        pred, u = int(rng.integers(0, MAX_K)), int(rng.integers(0, MAX_K))
        assert relax(pack(dist, edges, pred), delta, u) == pack(dist + delta, edges + 1, u)


def test_a_walk_one_edge_too_long_only_grows():
    """At edges = 2047 the edge count carries into the distance field: the
    candidate is then larger than the true extension, never smaller."""
    for dist, delta in [(0, 0), (-5, 3), (DMAX - 2**30, 2**30 - 1)]:
        c = relax(pack(dist, MAX_K - 1, 7), delta, 3)
        assert c > pack(dist + delta, MAX_K - 1, 3)
