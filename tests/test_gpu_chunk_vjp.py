"""The chunked family's IFT VJP reads only the active rows of J.

Every row-level term of eq. 17 carries the active set A*: an inactive row has
arefbar = Dbar = 0 and Jbar_i = -(0 lambda + 0 a), and adds nothing to the
refinement's J^T (D o A* o J v).  This checks, on uniform FP32 and FP64
batches solved by the chunked family, that the inactive rows' outputs are
exactly zero and that every output agrees with the generic team family's
VJP, which reads all rows, on the same saved state.
"""
import numpy as np
import pytest
import torch

from paper_2607_24959_amd import solver, synth
from paper_2607_24959_amd import _native as N

pytestmark = pytest.mark.gpu

KEYS = ("M", "J", "a0", "aref", "D", "abar")


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("dtype,n,nc", [(torch.float32, 40, 48), (torch.float32, 96, 96),
                                        (torch.float64, 24, 32)])
def test_chunk_vjp_reads_active_rows_only(dtype, n, nc):
    _needs_gpu()
    B, m = 96, 4 * nc
    hb = synth.uniform_batch(B, n, nc, seed=4242 + n)
    npd = np.float32 if dtype == torch.float32 else np.float64
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(hb, k).astype(npd))).cuda() for k in KEYS}
    bc = solver.Batch.uniform(B, n, m, dtype, path=N.PATH_CHUNK)
    sol = solver.forward(bc, t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=60,
                         tol=1e-5 if dtype == torch.float32 else 1e-12)
    gc = solver.ift_vjp(bc, sol, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"])
    # the team family's VJP on the same state (every family reads every family's state)
    bt = solver.Batch.uniform(B, n, m, dtype, path=N.PATH_TEAM)
    gt = solver.ift_vjp(bt, sol, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"])
    torch.cuda.synchronize()
    act = bc.active_sets(sol).reshape(B, m)
    assert 0 < act.mean() < 1, act.mean()
    a0b, arb, Jb, Db, Mb = (g.cpu().numpy() for g in gc)
    arb, Db, Jb = arb.reshape(B, m), Db.reshape(B, m), Jb.reshape(B, m, n)
    inact = ~act
    assert np.all(arb[inact] == 0) and np.all(Db[inact] == 0)
    assert np.all(Jb[inact] == 0)
    rtol = 2e-4 if dtype == torch.float32 else 1e-10
    for name, x, y in zip(("a0bar", "arefbar", "Jbar", "Dbar", "Mbar"), gc, gt):
        x, y = x.double().cpu().numpy().reshape(B, -1), y.double().cpu().numpy().reshape(B, -1)
        err = np.linalg.norm(x - y, axis=1) / np.maximum(np.linalg.norm(y, axis=1), 1e-30)
        assert np.max(err) <= rtol, (name, float(np.max(err)))
