"""Malformed packed descriptors on the GPU (the guarded path of every kernel
family): an instance whose offsets run past the batch's totals, one whose n
exceeds nv_max, and an order[] entry outside [0, B).  The malformed instances
get CS_ST_BADDESC (the out-of-range order entry: nothing), their outputs stay
untouched, and every other instance's results equal a clean run's bitwise."""
import numpy as np
import pytest
import torch

from paper_2607_24959_amd import _native as N
from paper_2607_24959_amd import solver, synth

pytestmark = pytest.mark.gpu

KEYS = ("M", "J", "a0", "aref", "D", "abar")
SENT = 12345.0


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(batch, t, prefill):
    s = batch.sizes()
    dt = batch.dtype
    sol = solver.Solution(a=torch.full((s["a"],), SENT, dtype=dt, device="cuda"),
                          state=torch.zeros(batch.state_bytes(), dtype=torch.uint8, device="cuda"),
                          status=torch.full((batch.B,), -7, dtype=torch.int32, device="cuda"),
                          iters=torch.full((batch.B,), -7, dtype=torch.int32, device="cuda"))
    solver.forward(batch, *(t[k] for k in KEYS[:5]), max_iter=40,
                   tol=1e-5 if dt == torch.float32 else 1e-12, out=sol)
    like = (t["a0"], t["aref"], t["J"], t["D"], t["M"])
    grads = tuple(torch.full_like(x, SENT) for x in like)
    solver.ift_vjp(batch, sol, *(t[k] for k in KEYS[:5]), t["abar"], out=grads)
    torch.cuda.synchronize()
    return sol, grads


@pytest.mark.parametrize("path,ns,dtype", [
    (N.PATH_SMALL, (3, 9), torch.float32), (N.PATH_WAVE, (9, 18, 31), torch.float32),
    (N.PATH_CHUNK, (18, 36, 96), torch.float32), (N.PATH_TEAM, (3, 18, 36), torch.float32),
    (N.PATH_SMALL, (3, 6), torch.float64), (N.PATH_CHUNK, (9, 24), torch.float64)])
def test_malformed_descriptor_is_skipped(path, ns, dtype):
    _needs_gpu()
    nc_max = 16 if path == N.PATH_SMALL else 64
    pb = synth.uneven_batch(40, ns, nc_max, seed=606, nc_min=1)
    npd = np.float32 if dtype == torch.float32 else np.float64
    px = pb.astype(npd)
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(px, k))).cuda() for k in KEYS}
    clean = solver.Batch.packed_from(pb.nv, pb.nrows, dtype, path=path)
    sol0, g0 = _run(clean, t, True)
    bad = solver.Batch.packed_from(pb.nv, pb.nrows, dtype, path=path)
    nv_d, nr_d, off_nn, off_mn, off_n, off_m = bad._keep[:6]
    off_mn[5] = bad.total_mn                 # J of instance 5 past the end
    nv_d[11] = bad.nv_max + 1                # instance 11 larger than the launch was sized for
    order = torch.arange(40, dtype=torch.int32, device="cuda")
    order[7] = 47                            # slot 7 names no instance
    bad.desc.order = order.data_ptr()
    bad._keep.append(order)
    torch.cuda.synchronize()
    sol1, g1 = _run(bad, t, True)
    st = sol1.status.cpu().numpy()
    assert st[5] == N.ST_BADDESC and st[11] == N.ST_BADDESC, st[[5, 11]]
    assert st[7] == -7                       # never processed
    a0, a1 = sol0.a.cpu().numpy(), sol1.a.cpu().numpy()
    offs = dict(a=pb.off_n, a0=pb.off_n, aref=pb.off_m, J=pb.off_mn, D=pb.off_m, M=pb.off_nn)
    for i in range(40):
        sl = slice(pb.off_n[i], pb.off_n[i + 1])
        if i in (5, 7, 11):
            assert np.all(a1[sl] == SENT), i
            continue
        assert st[i] == sol0.status.cpu().numpy()[i], i
        assert np.array_equal(a1[sl], a0[sl]), i
    for k, x0, x1 in zip(("a0", "aref", "J", "D", "M"), g0, g1):
        x0, x1 = x0.cpu().numpy(), x1.cpu().numpy()
        o = offs[k]
        for i in range(40):
            sl = slice(o[i], o[i + 1])
            if i in (5, 7, 11):
                assert np.all(x1[sl] == SENT), (k, i)
            else:
                assert np.array_equal(x1[sl], x0[sl]), (k, i)
