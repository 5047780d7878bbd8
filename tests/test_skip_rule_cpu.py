"""The solve kernel's exact skip of Negative Cycle Refinement, checked on the
CPU against the oracle's search.

After an allotment only row s of the best-transfer table can drop.  The
kernel keeps node potentials pot with pot[u] + W[u][v] >= pot[v] on every
edge (labels of an earlier search).  If no lowered entry of row s breaks that
inequality, the potentials still certify every cycle as non-negative, so the
search of Algorithm 1 from s cannot find a negative cycle and is skipped.
This test lowers random entries of row s of tables that carry such
potentials and, whenever the rule says skip, asks the oracle's search: it
must find no negative s_out -> s_in path."""
import numpy as np
import pytest

import oracle
from tests import pins


def _key(d, rank):
    return np.uint64(((int(d) + 2**31) << 32) | int(rank))


def _delta(key):
    return int(key >> np.uint64(32)) - 2**31


def _lowered_table(seed):
    """A table carrying the potentials pot, then random entries of row s
    lowered; breaks says whether a lowered entry breaks pot."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(2, 9))
    pot = rng.integers(-10, 11, size=k)
    W = np.full((k, k), pins.KEY_NONE, np.uint64)
    for u in range(k):
        for v in range(k):
            if u != v and rng.random() < 0.7:
                W[u, v] = _key(pot[v] - pot[u] + rng.integers(0, 4), rng.integers(0, 99))
    s = int(rng.integers(0, k))
    breaks = False
    for w in range(k):
        if w == s or rng.random() < 0.5:
            continue
        old = _delta(W[s, w]) if W[s, w] != pins.KEY_NONE else int(pot[w] - pot[s]) + 4
        new = old - int(rng.integers(0, 6))
        W[s, w] = _key(new, rng.integers(0, 99))
        breaks |= pot[s] + new < pot[w]
    z = np.zeros(k, np.int32)
    dist, _, _ = oracle.refine_search(W, s, 0, z, z, np.ones(k, np.int32))
    negative = dist[k] != oracle.DIST_NONE and dist[k] < 0
    return breaks, negative


@pytest.mark.parametrize("seed", range(200))
def test_skip_only_when_no_negative_cycle_is_possible(seed):
    breaks, negative = _lowered_table(seed)
    if not breaks:
        assert not negative, seed


def test_the_rule_is_not_vacuous():
    """Across the seeds both outcomes occur: some lowered rows keep the
    potentials, and some break them and hide a negative cycle."""
    outcomes = [_lowered_table(seed) for seed in range(200)]
    assert sum(not b for b, _ in outcomes) >= 10
    assert sum(b and n for b, n in outcomes) >= 10
