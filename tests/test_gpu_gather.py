"""fsda_gather_sum, the gather-rate measurement aid: its per-block sums add up
to the sum of src[idx] (tolerance from the summation order only)."""
import numpy as np
import pytest

import paper_1709_04794_amd as fsda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("size,nidx,grid", [(1000, 0, 4), (1000, 1, 1), (4096, 100003, 64), (200000, 1 << 20, 2048)])
def test_gather_sum_matches_indexing(size, nidx, grid):
    import torch
    rng = np.random.default_rng(size + nidx)
    src = torch.from_numpy(rng.standard_normal(size)).cuda()
    idx = torch.from_numpy(rng.integers(0, size, nidx).astype(np.int32)).cuda()
    part = fsda.gather_sum(src, idx, grid=grid)
    assert part.shape == (grid,)
    want = float(src.cpu().numpy()[idx.cpu().numpy()].sum()) if nidx else 0.0
    got = float(part.sum())
    assert abs(got - want) <= 1e-12 * max(1.0, float(np.abs(src.cpu().numpy()).sum()) * max(nidx, 1) / size)


def test_gather_sum_rejects_out_of_range_indices():
    import torch
    src = torch.zeros(10, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        fsda.gather_sum(src, torch.tensor([3, 10], dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError):
        fsda.gather_sum(src, torch.tensor([-1], dtype=torch.int32, device="cuda"))


def test_gather_sum_reuses_output_buffer():
    import torch
    src = torch.arange(100, dtype=torch.float64, device="cuda")
    idx = torch.arange(100, dtype=torch.int32, device="cuda")
    part = torch.full((8,), 7.0, dtype=torch.float64, device="cuda")
    out = fsda.gather_sum(src, idx, grid=8, part=part, checked=True)
    assert out.data_ptr() == part.data_ptr()
    assert float(out.sum()) == 4950.0
