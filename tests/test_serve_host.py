"""Host-side rules of the serving engine (no GPU): slot sizing from an HBM
budget, the slot table handed to the library, kernel classes and request
validation."""
import numpy as np
import pytest
import torch

from paper_2607_24959_amd import _native as N
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


def test_slot_table_layout():
    e = serve.Engine(slots=4, n_cap=9, m_cap=64, window=3, device="cpu")
    t = e.table
    assert (t.slots, t.window, t.n_cap, t.m_cap) == (4, 3, 9, 64)
    assert t.state == e.sol.state.data_ptr() and t.a == e.sol.a.data_ptr()
    # factors of the slot batch end before the active-set bytes, which fit the state
    ne = 9 * 10 // 2
    assert 4 * 4 * ne <= t.mask_offset
    assert t.mask_offset + 4 * 64 <= e.sol.state.numel()
    assert e.arch_fac.shape == (3, 4, ne) and e.arch_mask.shape == (3, 4, 64)


def test_kernel_classes():
    e32 = serve.Engine(slots=2, device="cpu")
    c = e32.classes
    assert e32.class_of(3, 0) != e32.class_of(9, 64)
    assert c[e32.class_of(9, 64)][0] == N.PATH_SMALL
    assert c[e32.class_of(9, 68)][0] == N.PATH_WAVE
    assert c[e32.class_of(18, 8)][0] == N.PATH_WAVE
    assert c[e32.class_of(18, 8)] != c[e32.class_of(9, 68)]   # padded widths 32 and 16
    e_wide = serve.Engine(slots=2, m_cap=1024, device="cpu")
    assert e_wide.classes[e_wide.class_of(18, 600)][0] == N.PATH_WAVE
    e_huge = serve.Engine(slots=2, m_cap=2048, device="cpu")
    assert e_huge.classes[e_huge.class_of(18, 1500)][0] == N.PATH_CHUNK
    assert e_wide.classes[e_wide.class_of(18, 100)][0] == N.PATH_WAVE
    e64 = serve.Engine(slots=2, dtype=torch.float64, device="cpu")
    assert e64.classes[e64.class_of(9, 8)][0] == N.PATH_CHUNK
    assert e64.classes[e64.class_of(6, 8)][0] == N.PATH_SMALL


def test_pool_and_request_checks():
    pool = serve.RequestPool(8, (3, 9), 16, 4, 3, 9, 64, torch.float64, "cpu")
    assert set(np.unique(pool.n)) <= {3, 9}
    assert np.all(pool.m == 4 * pool.nc) and pool.m.max() <= 64
    for i in range(8):
        n, m = int(pool.n[i]), int(pool.m[i])
        Mt = pool.Mt[i, :n * n].reshape(n, n)
        assert torch.equal(Mt, pool.Mp[i, :n, :n])
        assert torch.allclose(pool.Minv[i, :n * n].reshape(n, n) @ Mt, torch.eye(n, dtype=torch.float64))
        assert torch.equal(pool.Jt[i, :m * n].reshape(m, n), pool.Jp[i, :m, :n])
        assert torch.count_nonzero(pool.Mt[i, n * n:]) == 0
    e = serve.Engine(slots=2, n_cap=9, m_cap=32, window=4, dtype=torch.float64, device="cpu")
    with pytest.raises(ValueError):
        e.attach_pool(pool)
    with pytest.raises(ValueError):
        e.submit(serve.Request(rid=0, pool_index=0, n=9, m=64))
    with pytest.raises(ValueError):
        serve.RequestPool(4, (12,), 4, 4, 3, 9, 64, torch.float64, "cpu")


def test_serve_entry_points_reject_bad_tables():
    e = serve.Engine(slots=2, n_cap=9, m_cap=64, window=3, device="cpu")
    bad = N.CsServeTable()
    assert N.serve_pre(bad, None, 0, None) == N.CS_EINVAL
    assert N.serve_post(bad, None, 0, None) == N.CS_EINVAL
    assert N.serve_pre(e.table, None, 1, None) == N.CS_EINVAL       # entries required
    assert N.serve_pre(e.table, None, -1, None) == N.CS_EINVAL
    assert N.serve_pre(e.table, None, 0, None) == N.CS_OK            # nothing to do
    pool = serve.RequestPool(2, (9,), 16, 3, 1, 9, 64, torch.float32, "cpu")
    assert N.serve_admit(e.table, pool.table, None, 0, None) == N.CS_OK
    pool64 = serve.RequestPool(2, (9,), 16, 3, 1, 9, 64, torch.float64, "cpu")
    assert N.serve_admit(e.table, pool64.table, None, 0, None) == N.CS_EINVAL   # dtype differs
    t = N.CsServeTable.from_buffer_copy(e.table)
    t.n_cap = 65
    assert N.serve_pre(t, None, 0, None) == N.CS_EINVAL


def test_serve_tick_rejects_bad_arguments():
    """cs_serve_tick checks every argument before it enqueues anything (no
    device is touched: each case fails a check, and the device list address
    below is never dereferenced)."""
    if torch.cuda.is_available():
        pytest.skip("host argument checks only, with a placeholder device address")
    e = serve.Engine(slots=2, n_cap=9, m_cap=64, window=3, device="cpu")
    rows = np.zeros((2, 5), dtype=np.int32)
    host = np.zeros(16, dtype=np.int32)
    dev_list = 0x1000

    def tick(table=None, pool=None, ncls=None, list_len=16, n_admit=0, n_entries=1, nl=1,
             host_ptr=host.ctypes.data, side=None):
        return N.serve_tick(e.table if table is None else table, pool, e.class_arr,
                            len(e.classes) if ncls is None else ncls, e.params, 0, None, None,
                            host_ptr, dev_list, list_len, n_admit, n_entries, rows.ctypes.data,
                            nl, None, side, None, None, None)

    rows[0] = (0, 0, 0, 1, 2)                     # a forward of class 0 on lane 0
    assert tick(table=N.CsServeTable()) == N.CS_EINVAL
    assert tick(ncls=0) == N.CS_EINVAL
    assert tick(list_len=2) == N.CS_EINVAL        # the launch's order lies past the list
    assert tick(list_len=-1) == N.CS_EINVAL
    assert tick(host_ptr=None) == N.CS_EINVAL
    assert tick(n_admit=1) == N.CS_EINVAL         # admission needs the pool table
    assert tick(n_entries=-1) == N.CS_EINVAL
    assert tick(nl=-1) == N.CS_EINVAL
    for bad in ((2, 0, 0, 1, 2),                  # kind
                (0, len(e.classes), 0, 1, 2),     # class index
                (0, -1, 0, 1, 2),
                (0, 0, 2, 1, 2),                  # lane
                (0, 0, 0, 0, 2),                  # empty launch
                (0, 0, 0, 15, 2),                 # order + count past the list
                (0, 0, 0, 1, -1),
                (1, 0, 1, 1, 2)):                 # lane 1 without a side stream and events
        rows[0] = bad
        assert tick() == N.CS_EINVAL, bad
    rows[0] = (0, 0, 0, 1, 2)
    rows[1] = (1, 0, 1, 1, 3)
    assert tick(nl=2) == N.CS_EINVAL              # side lane named, side stream missing


def test_deal_lanes_orders_and_balances():
    """Longest launches first (forwards by class width, VJPs shortest), each
    to the less loaded lane; one lane when the tick has no second lane."""
    classes = [(N.PATH_SMALL, 3, 64), (N.PATH_SMALL, 9, 64), (N.PATH_WAVE, 15, 256),
               (N.PATH_WAVE, 18, 256)]
    rows = np.zeros((8, 5), dtype=np.int32)
    launches = [("vjp", 3, 10, 2), ("fwd", 0, 12, 3), ("fwd", 3, 15, 1), ("fwd", 2, 16, 4),
                ("vjp", 0, 20, 1)]
    out = serve.deal_lanes(list(launches), classes, True, rows)
    # estimates: fwd c3 76, fwd c2 70, fwd c0 46, vjp 20, vjp 20
    assert [tuple(r) for r in out] == [(0, 3, 0, 1, 15), (0, 2, 1, 4, 16), (0, 0, 1, 3, 12),
                                       (1, 3, 0, 2, 10), (1, 0, 0, 1, 20)]
    out1 = serve.deal_lanes(list(launches), classes, False, rows)
    assert set(out1[:, 2].tolist()) == {0}
    assert sorted(map(tuple, out1[:, [0, 1, 3, 4]].tolist())) == \
        sorted((0 if k == "fwd" else 1, c, n, o) for k, c, o, n in launches)
