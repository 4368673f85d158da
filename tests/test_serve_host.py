"""Host-side rules of the serving engine (no GPU): slot sizing from an HBM
budget and request validation."""
import numpy as np
import pytest
import torch

from paper_2607_24959_amd import serve


def test_slots_follow_budget():
    per = serve.slot_bytes(18, 256, 6, 4)
    assert per > 0 and serve.slot_bytes(18, 256, 6, 8) > per
    e = serve.Engine(budget_bytes=7 * per + 1, device="cpu")
    assert e.S == 7
    with pytest.raises(ValueError):
        serve.Engine(budget_bytes=per - 1, device="cpu")
    with pytest.raises(ValueError):
        serve.Engine(device="cpu")


def test_slot_layout_views():
    e = serve.Engine(slots=4, n_cap=9, m_cap=64, device="cpu")
    ne = 9 * 10 // 2
    assert e.fac_view.shape == (4, ne)
    assert e.mask_view.shape == (4, 64)
    # the factor and mask views lie inside the state buffer, disjoint
    assert e.fac_view.numel() * 4 <= e.batch.mask_offset()
    assert e.batch.mask_offset() + 4 * 64 <= e.sol.state.numel()


def test_pool_and_request_checks():
    pool = serve.RequestPool(8, (3, 9), 16, 4, 3, 9, 64, torch.float64, "cpu")
    assert set(np.unique(pool.n)) <= {3, 9}
    assert np.all(pool.m == 4 * pool.nc) and pool.m.max() <= 64
    for i in range(8):
        n, m = int(pool.n[i]), int(pool.m[i])
        Mt = pool.Mt[i, :n * n].reshape(n, n)
        assert torch.equal(Mt, pool.Mp[i, :n, :n])
        assert torch.equal(pool.Jt[i, :m * n].reshape(m, n), pool.Jp[i, :m, :n])
        assert torch.count_nonzero(pool.Mt[i, n * n:]) == 0
    e = serve.Engine(slots=2, n_cap=9, m_cap=32, window=4, device="cpu")
    with pytest.raises(ValueError):
        e.attach_pool(pool)
    with pytest.raises(ValueError):
        e.submit(serve.Request(rid=0, pool_index=0, n=9, m=64))
