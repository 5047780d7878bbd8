"""lbdd_best_transfers_noalloc against lbdd_best_transfers, bit-exact.

The no-allocation entry point takes its workspace from the library's fixed
per-GPU scratch; its table must equal the table of the entry point that takes
a workspace argument, on two calls in a row (the second with a smaller
input, so the scratch holds the first call's leftovers), and calls beyond
the scratch's size are refused with an error before any launch."""
import sys

import numpy as np
import pytest

import lbdd_inputs as L

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lb():
    import torch
    import paper_2304_06543_amd.lbdd as lb
    lb.load()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lb


def _inputs(inst, seed):
    import torch
    rng = np.random.default_rng(seed)
    cm = torch.from_numpy(inst.cm).cuda()
    a = torch.from_numpy(rng.integers(0, inst.k, size=inst.n).astype(np.int32)).cuda()
    r = torch.from_numpy(rng.permutation(inst.n).astype(np.int32)).cuda()
    return cm, a, r


def test_noalloc_equals_workspace_entry_point(lb):
    import torch
    cases = [L.gmm_manhattan(100, 200_000, seed=71, cap_frac=0.95, pen_lo=100, pen_hi=1000),
             L.random_small(k=37, n=5003, seed=72, cm_hi=900)]
    for j, inst in enumerate(cases):
        say("noalloc scan", inst.k, inst.n)
        cm, a, r = _inputs(inst, 500 + j)
        ref = lb.best_transfers(cm, a, r)
        W = torch.full((inst.k, inst.k), 7, dtype=torch.int64, device="cuda")
        lb.best_transfers_noalloc(cm, a, r, W)
        torch.cuda.synchronize()
        assert torch.equal(W, ref), j
        # the grouping this call left in the scratch serves a rescan
        W2 = torch.zeros_like(W)
        lb.best_transfers_noalloc(cm, a, r, W2, reuse_grouping=True)
        torch.cuda.synchronize()
        assert torch.equal(W2, ref), j


def test_noalloc_refuses_sizes_beyond_the_scratch(lb):
    import torch
    k, n = 8, 3_000_000
    assert lb.best_transfers_work_bytes(k, n) > lb.NOALLOC_SCRATCH_BYTES
    cm = torch.zeros((1, k), dtype=torch.int32, device="cuda")   # never read: the size check comes first
    W = torch.empty((k, k), dtype=torch.int64, device="cuda")
    lib = lb.load()
    import ctypes as C
    p = C.c_void_p(cm.data_ptr())
    rc = lib.lbdd_best_transfers_noalloc(k, n, p, p, p, C.c_void_p(W.data_ptr()), 0, None)
    assert rc == lb.E_INVAL
    assert b"scratch" in lib.lbdd_last_error()
