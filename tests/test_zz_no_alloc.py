"""The allocation-free segmented sort (bitonic_sort_segmented_noalloc_i32)
against the allocating entry point it is a variant of
(bitonic_sort_segmented_bounded_i32) and the oracle, bit for bit, on two
calls in a row, the second with a smaller table."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1506_01446_amd import binding as B
from paper_1506_01446_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load()


def _case(nseg, seed, max_log2):
    lens = W.segment_lengths(seed, nseg, max_log2)
    lens[:4] = [0, 1, 8193, 2 ** int(max_log2)]  # empty, one key, first big class, the bound
    off = W.offsets_from_lengths(lens) + 3       # unaligned start, offsets[0] != 0
    keys = W.uniform_i32(seed + 1, int(off[-1]) + 5)
    return keys, off, int(lens.max())


@pytest.mark.parametrize("asc", [True, False])
def test_noalloc_matches_bounded_two_calls(asc):
    cases = [(3000, W.SEED_BASE + 60, 16.0), (700, W.SEED_BASE + 62, 14.0)]
    for nseg, seed, max_log2 in cases:
        keys, off, bound = _case(nseg, seed, max_log2)
        print(f"[case] noalloc nseg={nseg} keys={off[-1]} bound={bound} asc={asc}", flush=True)
        o = torch.from_numpy(off).cuda()
        a = torch.from_numpy(keys.copy()).cuda()
        b = torch.from_numpy(keys.copy()).cuda()
        B.bitonic_sort_segmented_noalloc_i32(a, o, bound, asc)
        B.bitonic_sort_segmented_i32(b, o, asc, max_seg_len=bound)
        torch.cuda.synchronize()
        got, ref = a.cpu().numpy(), b.cpu().numpy()
        assert np.array_equal(got, ref), (nseg, asc)
        assert np.array_equal(got, O.sort_segmented_i32(keys, off, asc)), (nseg, asc)


def test_noalloc_limits():
    """Tables past the array's capacity are refused before anything runs."""
    k = torch.zeros(8, dtype=torch.int32, device="cuda")
    big = torch.zeros((1 << 18) + 1, dtype=torch.int64, device="cuda")  # 2^18 segments
    with pytest.raises(B.BitonicError) as e:
        B.bitonic_sort_segmented_noalloc_i32(k, big, 8)
    assert e.value.status == -4
    o = torch.tensor([0, 8], dtype=torch.int64, device="cuda")
    with pytest.raises(B.BitonicError) as e:
        B.bitonic_sort_segmented_noalloc_i32(k, o, 0)  # a bound is required
    assert e.value.status == -1
