"""The read-only streaming kernel behind the bandwidth ceiling
(lbdd_read_ceiling): it must read every byte it is given, which its XOR fold
shows, for any workgroup count and any size that is a multiple of 16."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    import paper_2304_06543_amd.lbdd as lb
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lb.load()
    return lb


@pytest.mark.parametrize("words,blocks", [(4, 1), (4, 7), (1000, 3), (4096, 256), (262148, 1024),
                                          (1 << 22, 256), ((1 << 22) + 12, 4096)])
def test_fold_covers_every_word(lb, words, blocks):
    import torch
    rng = np.random.default_rng(words + blocks)
    a = rng.integers(0, 1 << 32, size=words, dtype=np.uint64).astype(np.uint32)
    buf = torch.from_numpy(a.view(np.int32)).cuda()
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    lb.read_ceiling(buf, sink, blocks)
    torch.cuda.synchronize()
    assert int(sink.item()) == int(np.bitwise_xor.reduce(a))
    # a second call folds the same value in again
    lb.read_ceiling(buf, sink, blocks)
    torch.cuda.synchronize()
    assert int(sink.item()) == 0


def test_bad_arguments_are_refused(lb):
    import torch
    buf = torch.zeros(8, dtype=torch.int32, device="cuda")
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(lb.LbddError):
        lb.read_ceiling(buf[:3], sink, 4)          # 12 bytes: not a multiple of 16
    with pytest.raises(lb.LbddError):
        lb.read_ceiling(buf, sink, 0)
