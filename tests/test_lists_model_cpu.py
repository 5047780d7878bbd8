"""The solve kernel's bounded best-transfer lists, modelled on the CPU.

Gamma (Section 3.2) needs, per ordered center pair (u, w), the smallest
transfer key over the units currently at u; the paper keeps a heap per pair
(the BestTransHeap of Section 3.5).  The kernel keeps only a sorted list of at
most BEST_M keys per pair, a count c, an every-unit-held flag, and a
threshold below which a joining key enters; a list that runs empty while
some unit of u is not in it is refilled by a scan of u's members.

The claim that makes the list head exact: while a list is not empty-and-
incomplete it holds exactly the c smallest keys of the center's members (all
of them when the flag is set).  This model applies the kernel's merge,
threshold and removal rules to random join/leave sequences and checks that
claim, and the head against the true minimum, after every step."""
import numpy as np
import pytest

NONE = 2**64 - 1
M = 8


def merge(a, q):
    """The sorted list with q merged in; the largest entry falls off."""
    return sorted(a + [q])[:M]


def threshold(a, c, every):
    if every:
        return NONE                              # every key enters
    return a[c - 1] if c > 0 else 0              # in front of the last held key


class PairList:
    def __init__(self):
        self.a, self.c, self.every = [NONE] * M, 0, True
        self.thr = threshold(self.a, 0, True)

    def join(self, q):
        if not q < self.thr:
            return
        full = self.c == M
        self.a = merge(self.a, q)
        self.c = M if full else self.c + 1
        self.every = self.every and not full
        self.thr = threshold(self.a, self.c, self.every)

    def leave(self, q):
        if q not in self.a:
            return                               # not among the c smallest
        i = self.a.index(q)
        self.a = self.a[:i] + self.a[i + 1:] + [NONE]
        self.c -= 1
        self.thr = threshold(self.a, self.c, self.every)

    def unknown(self):
        return self.c == 0 and not self.every

    def refill(self, members):
        keys = sorted(members)[:M]
        self.a = keys + [NONE] * (M - len(keys))
        self.c = len(keys)
        self.every = len(members) <= M
        self.thr = threshold(self.a, self.c, self.every)


@pytest.mark.parametrize("seed", range(40))
def test_lists_hold_the_smallest_keys_after_every_step(seed):
    rng = np.random.default_rng(seed)
    pool = [int(x) for x in rng.choice(10**6, size=300, replace=False)]
    members, L = set(), PairList()
    for step in range(600):
        outside = [q for q in pool if q not in members]
        # bias toward joins early and leaves late so lists fill, overflow and drain
        p_join = 0.8 if step < 200 else 0.35
        if members and (not outside or rng.random() > p_join):
            q = sorted(members)[int(rng.integers(0, len(members)))]
            members.discard(q)
            L.leave(q)
        else:
            q = outside[int(rng.integers(0, len(outside)))]
            members.add(q)
            L.join(q)
        if L.unknown():
            L.refill(members)
        truth = sorted(members)
        assert L.a[:L.c] == truth[:L.c], (seed, step)
        if L.every:
            assert L.c == len(truth)
        head = L.a[0] if L.c else NONE
        assert head == (truth[0] if truth else NONE), (seed, step)


def test_threshold_rejects_keys_beyond_the_last_held_one():
    L = PairList()
    for q in range(100, 100 + 2 * M):            # overflow: the flag clears
        L.join(q)
    assert L.c == M and not L.every
    L.join(500)                                  # beyond the last held key
    assert L.a == list(range(100, 100 + M))
    L.join(50)                                   # in front: enters, the largest drops
    assert L.a == [50] + list(range(100, 100 + M - 1))


def test_a_drained_list_is_refilled_from_the_members():
    L, members = PairList(), set(range(100, 100 + 2 * M))
    for q in sorted(members):
        L.join(q)
    for q in range(100, 100 + M):                # the held keys leave
        members.discard(q)
        L.leave(q)
    assert L.unknown()                           # empty, yet units remain
    L.refill(members)
    assert L.a == sorted(members) and L.every and L.c == M
