"""Batched solve (one persistent launch for many instances) against the
oracle and against plain one-instance solves, bit-exact."""
import sys

import numpy as np
import pytest

import lbdd_inputs as L
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lb():
    import torch
    import paper_2304_06543_amd.lbdd as lb
    lb.load()
    assert torch.cuda.is_available()
    return lb


def mixed_instances(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        k = int(rng.choice([1, 3, 8, 17, 37, 64, 100, 133, 140, 250]))
        n = int(rng.integers(1, 900))
        out.append(L.random_small(k=k, n=n, seed=1000 * seed + j, cm_hi=int(rng.choice([4, 80, 2000])),
                                  cap=["tight", "zero", "loose", 3][j % 4], pen_hi=300))
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_batch_matches_oracle(lb, seed):
    import torch
    insts = mixed_instances(24, seed)
    say("batch", seed, [(i.k, i.n) for i in insts])
    hs = [lb.Instance(torch.from_numpy(i.cm).cuda(), i.cap, i.pen) for i in insts]
    lb.solve_batch(hs)
    for inst, h in zip(insts, hs):
        ref = oracle.solve(*inst.arrays())
        assert h.objective() == ref.objective, inst.name
        assert np.array_equal(h.assignment(), ref.assign), inst.name
        h.close()


def test_batch_continues_partial_and_skips_solved(lb):
    import torch
    insts = mixed_instances(6, 7)
    hs = [lb.Instance(torch.from_numpy(i.cm).cuda(), i.cap, i.pen) for i in insts]
    hs[0].solve_iters(5)
    hs[1].solve()
    hs[2].solve_iters(insts[2].n // 2)
    lb.solve_batch(hs)
    for inst, h in zip(insts, hs):
        ref = oracle.solve(*inst.arrays())
        assert h.progress() == inst.n
        assert h.objective() == ref.objective and np.array_equal(h.assignment(), ref.assign)
        h.close()


def test_batch_on_its_own_stream(lb):
    import torch
    insts = mixed_instances(5, 9)
    side = torch.cuda.Stream()
    hs = [lb.Instance(torch.from_numpy(i.cm).cuda(), i.cap, i.pen) for i in insts]
    lb.solve_batch(hs, stream=side)
    for inst, h in zip(insts, hs):
        ref = oracle.solve(*inst.arrays())
        assert h.objective() == ref.objective and np.array_equal(h.assignment(), ref.assign)
        h.close()


def test_batch_rejects_bad_lists(lb):
    import torch
    i = L.random_small(k=3, n=10, seed=1)
    h = lb.Instance(torch.from_numpy(i.cm).cuda(), i.cap, i.pen)
    with pytest.raises(lb.LbddError):
        lb.solve_batch([h, h])
    lb.solve_batch([])
    h.close()
