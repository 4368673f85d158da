"""Mixed regularised rows on the GPU (cs_forward_rows, cs_ift_vjp_rows):
pyramid contact rows, equality rows and friction-loss rows against the oracle,
instance by instance.

* FP64: a within 1e-10, every row's zone code and the status equal, the VJP
  (a0, aref, J, D, floss, M) within 1e-8;
* FP32 storage (FP64 arithmetic inside): a within 1e-5 and the zones equal,
  except instances the oracle finds with a row within 1e-7 (relative) of a
  zone boundary; the VJP within 1e-3 of the oracle's and within 1e-5 of the
  oracle's at the GPU's own a;
* one-sided rows alone equal cs_forward (pyramid) to 1e-10; a bad kind gives
  ST_NONFINITE.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2607_24959_amd import solver, synth
from paper_2607_24959_amd import _native as N

pytestmark = pytest.mark.gpu

KEYS = ("M", "J", "a0", "aref", "D")
GK = ("a0", "aref", "J", "D", "floss", "M")


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _gpu(b, dtype, max_iter, tol, vjp=True):
    batch = solver.Batch.uniform(b.B, b.n, b.m, dtype)
    d = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)
    t = {k: d(getattr(b, k)) for k in KEYS + ("floss", "abar")}
    kind = torch.from_numpy(np.ascontiguousarray(b.kind)).cuda()
    sol = solver.forward_rows(batch, *(t[k] for k in KEYS), kind, t["floss"], max_iter=max_iter,
                              tol=tol)
    out = dict(a=sol.a.double().cpu().numpy(), status=sol.status.cpu().numpy(),
               zone=sol.state[batch.mask_offset():batch.mask_offset() + b.B * b.m].cpu().numpy()
               .reshape(b.B, b.m))
    if vjp:
        g = solver.ift_vjp_rows(batch, sol, *(t[k] for k in KEYS), kind, t["floss"], t["abar"])
        out.update({k: v.double().cpu().numpy() for k, v in g.items()})
    torch.cuda.synchronize()
    return out


def _rel(x, ref):
    x, ref = np.asarray(x).ravel(), np.asarray(ref).ravel()
    return np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300)


def _margin(b, i, a):
    r = b.J[i] @ a - b.aref[i]
    sc = np.abs(b.aref[i]) + np.abs(b.J[i]) @ np.abs(a) + 1e-300
    d = np.where(b.kind[i] == 0, np.abs(r),
                 np.where(b.kind[i] == 2, np.abs(np.abs(r) - b.floss[i] / b.D[i]), np.inf))
    return float((d / sc).min())


@pytest.mark.parametrize("B,n,nc,ne,nf", [(128, 6, 4, 2, 3), (64, 9, 16, 4, 8), (33, 18, 8, 3, 6)])
def test_fp64_matches_oracle(B, n, nc, ne, nf):
    _needs_gpu()
    b = synth.mixed_batch(B, n, nc, ne, nf, synth.SEED_BASE + 80 + n)
    g = _gpu(b, torch.float64, 80, 1e-12)
    for i in range(B):
        args = (b.M[i], b.J[i], b.a0[i], b.aref[i], b.D[i], b.kind[i], b.floss[i])
        o = oracle.forward_rows(*args, max_iter=80, tol=1e-12)
        assert o["status"] == oracle.ST_CONVERGED
        assert g["status"][i] == o["status"], i
        assert np.array_equal(g["zone"][i], o["zone"]), i
        assert _rel(g["a"][i], o["a"]) <= 1e-10, (i, _rel(g["a"][i], o["a"]))
        og = oracle.ift_vjp_rows(*args, o["a"], b.abar[i])
        for k in GK:
            if np.abs(og[k]).max() == 0:
                assert np.abs(g[k][i]).max() == 0, (i, k)
                continue
            assert _rel(g[k][i], og[k]) <= 1e-8, (i, k, _rel(g[k][i], og[k]))


def test_fp32_storage():
    _needs_gpu()
    b = synth.mixed_batch(512, 9, 16, 4, 8, synth.SEED_BASE + 90)
    b32 = b.astype(np.float32)
    br = b.rounded(np.float32)
    g = _gpu(b32, torch.float32, 80, 1e-7)
    excluded, wa, wg, ws = 0, 0.0, 0.0, 0.0
    for i in range(b.B):
        args = (br.M[i], br.J[i], br.a0[i], br.aref[i], br.D[i], br.kind[i], br.floss[i])
        o = oracle.forward_rows(*args, max_iter=80, tol=1e-12)
        assert o["status"] == oracle.ST_CONVERGED
        assert g["status"][i] & oracle.ST_CONVERGED, i
        if _margin(br, i, o["a"]) < 1e-7:
            excluded += 1
            continue
        assert np.array_equal(g["zone"][i], o["zone"]), i
        ea = _rel(g["a"][i], o["a"])
        wa = max(wa, ea)
        assert ea <= 1e-5, (i, ea)
        og = oracle.ift_vjp_rows(*args, o["a"], br.abar[i])
        sp = oracle.ift_vjp_rows(*args, g["a"][i], br.abar[i])
        for k in GK:
            if np.abs(og[k]).max() == 0:
                continue
            e, e2 = _rel(g[k][i], og[k]), _rel(g[k][i], sp[k])
            wg, ws = max(wg, e), max(ws, e2)
            assert e <= 1e-3, (i, k, e)
            assert e2 <= 1e-5, (i, k, e2)
    print(dict(excluded=excluded / b.B, a_max=wa, grad_max=wg, same_point_max=ws), flush=True)
    assert excluded / b.B < 0.01


def test_one_sided_rows_equal_the_pyramid_solver_and_bad_kind():
    _needs_gpu()
    b = synth.mixed_batch(64, 9, 16, 0, 0, 7)
    g = _gpu(b, torch.float64, 80, 1e-12, vjp=False)
    batch = solver.Batch.uniform(b.B, b.n, b.m, torch.float64)
    d = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda", torch.float64)
    sol = solver.forward(batch, *(d(getattr(b, k)) for k in KEYS), max_iter=80, tol=1e-12)
    torch.cuda.synchronize()
    a = sol.a.cpu().numpy()
    for i in range(b.B):
        assert _rel(g["a"][i], a[i]) <= 1e-10, i
    bb = synth.mixed_batch(8, 6, 2, 1, 1, 8)
    bb.kind[2, 0] = 7
    gb = _gpu(bb, torch.float64, 80, 1e-12, vjp=False)
    assert gb["status"][2] == N.ST_NONFINITE
    assert np.all(gb["status"][[0, 1, 3, 4, 5, 6, 7]] == N.ST_CONVERGED)
