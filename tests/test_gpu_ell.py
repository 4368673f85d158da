"""Round (elliptic) cone on the GPU (cs_forward_ell, cs_ift_vjp_ell) against
the oracle, instance by instance.

* FP64 uniform batches: a within 1e-10, every contact's zone and the status
  equal, the seven VJP outputs (a0, aref, J, D_N, D_T, mu, M) within 1e-8;
* FP64 packed batch of mixed shapes (n in {3, 9, 18, 32}, 0..40 contacts);
* FP32 storage (B=1024, n=9, 16 contacts; FP64 arithmetic inside): a within
  1e-5 and the zones equal, except instances the oracle finds with a contact
  within 1e-7 (relative) of a zone boundary; the VJP within 1e-3 of the
  oracle's and within 1e-5 of the oracle's at the GPU's own a;
* mu = 0 equals the pyramid solve on the normal rows; no contacts gives a0;
  non-finite input; argument errors.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2607_24959_amd import solver, synth
from paper_2607_24959_amd import _native as N

pytestmark = pytest.mark.gpu

KEYS = ("M", "J", "a0", "aref", "dn", "dt", "mu")
GK = ("a0", "aref", "J", "dn", "dt", "mu", "M")


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def _gpu(b, dtype, max_iter, tol, vjp=True):
    batch = solver.Batch.uniform(b.B, b.n, b.m, dtype)
    t = {k: _dev(getattr(b, k), dtype) for k in KEYS + ("abar",)}
    sol = solver.forward_ell(batch, *(t[k] for k in KEYS), max_iter=max_iter, tol=tol)
    out = dict(a=sol.a.double().cpu().numpy(), status=sol.status.cpu().numpy(),
               iters=sol.iters.cpu().numpy(),
               zone=batch.zones(sol).reshape(b.B, b.nc))
    if vjp:
        g = solver.ift_vjp_ell(batch, sol, *(t[k] for k in KEYS), t["abar"])
        out.update({k: v.double().cpu().numpy() for k, v in g.items()})
    torch.cuda.synchronize()
    return out


def _rel(x, ref):
    x, ref = np.asarray(x).ravel(), np.asarray(ref).ravel()
    return np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300)


def _margin(b, i, a):
    """Smallest relative distance of a contact's scaled residual from a zone boundary."""
    u = b.J[i] @ a - b.aref[i]
    best = np.inf
    for c in range(b.nc):
        sn, st = np.sqrt(b.dn[i][c]), np.sqrt(b.dt[i][c])
        mh = b.mu[i][c] * sn / st
        nn, t = sn * u[3 * c], st * np.hypot(u[3 * c + 1], u[3 * c + 2])
        sc = abs(nn) + mh * t + t + 1e-300
        best = min(best, abs(nn - mh * t) / sc, abs(mh * nn + t) / sc)
    return best


@pytest.mark.parametrize("B,n,nc", [(256, 6, 4), (128, 9, 16), (64, 18, 12), (37, 32, 20)])
def test_fp64_uniform_matches_oracle(B, n, nc):
    _needs_gpu()
    b = synth.elliptic_batch(B, n, nc, synth.SEED_BASE + 60 + n)
    g = _gpu(b, torch.float64, 80, 1e-12)
    iters_diff = 0
    for i in range(B):
        args = [getattr(b, k)[i] for k in KEYS]
        o = oracle.forward_ell(*args, max_iter=80, tol=1e-12)
        assert o["status"] == oracle.ST_CONVERGED
        assert g["status"][i] == o["status"], i
        assert np.array_equal(g["zone"][i], o["zone"]), i
        assert _rel(g["a"][i], o["a"]) <= 1e-10, (i, _rel(g["a"][i], o["a"]))
        iters_diff += int(g["iters"][i] != o["iters"])
        og = oracle.ift_vjp_ell(*args, o["a"], b.abar[i])
        for k in GK:
            e = _rel(g[k][i], og[k])
            assert e <= 1e-8, (i, k, e)
    print(dict(B=B, n=n, nc=nc, iters_differ=iters_diff, mean_iters=float(g["iters"].mean())),
          flush=True)


def test_fp64_packed_mixed_shapes():
    _needs_gpu()
    shapes = [(n, nc) for n in (3, 9, 18, 32) for nc in (0, 1, 7, 40)]
    inst = [synth.elliptic_batch(1, n, nc, 500 + k) for k, (n, nc) in enumerate(shapes)]
    nv = np.array([x.n for x in inst], np.int32)
    nrows = np.array([x.m for x in inst], np.int32)
    batch = solver.Batch.packed_from(nv, nrows, torch.float64)
    flat = {k: np.concatenate([getattr(x, k)[0].ravel() for x in inst]) for k in KEYS + ("abar",)}
    t = {k: _dev(v, torch.float64) for k, v in flat.items()}
    sol = solver.forward_ell(batch, *(t[k] for k in KEYS), max_iter=80, tol=1e-12)
    g = solver.ift_vjp_ell(batch, sol, *(t[k] for k in KEYS), t["abar"])
    torch.cuda.synchronize()
    a = sol.a.cpu().numpy()
    st = sol.status.cpu().numpy()
    on = np.concatenate([[0], np.cumsum(nv)])
    om = np.concatenate([[0], np.cumsum(nrows)])
    onn = np.concatenate([[0], np.cumsum(nv * nv)])
    omn = np.concatenate([[0], np.cumsum(nrows * nv)])
    oc = om // 3
    for i, x in enumerate(inst):
        args = [getattr(x, k)[0] for k in KEYS]
        o = oracle.forward_ell(*args, max_iter=80, tol=1e-12)
        assert st[i] == o["status"] == oracle.ST_CONVERGED, i
        assert _rel(a[on[i]:on[i + 1]], o["a"]) <= 1e-10, i
        og = oracle.ift_vjp_ell(*args, o["a"], x.abar[0])
        spans = dict(a0=(on, 1), aref=(om, 1), J=(omn, 1), dn=(oc, 1), dt=(oc, 1), mu=(oc, 1),
                     M=(onn, 1))
        for k in GK:
            off = spans[k][0]
            got = g[k].cpu().numpy()[off[i]:off[i + 1]]
            if og[k].size == 0 or np.asarray(og[k]).ravel().size == 0:
                continue
            assert _rel(got, og[k]) <= 1e-8 or np.abs(og[k]).max() == 0, (i, k)


def test_fp32_storage_b1024_n9_nc16():
    _needs_gpu()
    b = synth.elliptic_batch(1024, 9, 16, synth.SEED_BASE + 70)
    b32 = b.astype(np.float32)
    br = b.rounded(np.float32)
    g = _gpu(b32, torch.float32, 80, 1e-7)
    excluded, worst_a, worst_g, worst_sp = 0, 0.0, 0.0, 0.0
    for i in range(b.B):
        args = [getattr(br, k)[i] for k in KEYS]
        o = oracle.forward_ell(*args, max_iter=80, tol=1e-12)
        assert o["status"] == oracle.ST_CONVERGED
        assert g["status"][i] & oracle.ST_CONVERGED, i
        if _margin(br, i, o["a"]) < 1e-7:
            excluded += 1
            continue
        assert np.array_equal(g["zone"][i], o["zone"]), i
        ea = _rel(g["a"][i], o["a"])
        worst_a = max(worst_a, ea)
        assert ea <= 1e-5, (i, ea)
        og = oracle.ift_vjp_ell(*args, o["a"], br.abar[i])
        sp = oracle.ift_vjp_ell(*args, g["a"][i], br.abar[i])
        for k in GK:
            e = _rel(g[k][i], og[k])
            e2 = _rel(g[k][i], sp[k])
            worst_g, worst_sp = max(worst_g, e), max(worst_sp, e2)
            assert e <= 1e-3, (i, k, e)
            assert e2 <= 1e-5, (i, k, e2)
    print(dict(excluded=excluded / b.B, a_max=worst_a, grad_max=worst_g, same_point_max=worst_sp,
               mean_iters=float(g["iters"].mean())), flush=True)
    assert excluded / b.B < 0.01


def test_mu_zero_no_contacts_nonfinite_and_errors():
    _needs_gpu()
    b = synth.elliptic_batch(64, 6, 5, 91)
    b.mu[:] = 0.0
    g = _gpu(b, torch.float64, 80, 1e-12, vjp=False)
    for i in range(8):
        p = oracle.forward(b.M[i], b.J[i][0::3], b.a0[i], b.aref[i][0::3], b.dn[i], max_iter=80,
                           tol=1e-12)
        assert _rel(g["a"][i], p["a"]) <= 1e-10
        assert np.array_equal(g["zone"][i] != 0, p["active"])
    b0 = synth.elliptic_batch(8, 5, 0, 92)
    g0 = _gpu(b0, torch.float64, 80, 1e-12)
    assert np.array_equal(g0["a"], b0.a0) and np.all(g0["status"] == N.ST_CONVERGED)
    bn = synth.elliptic_batch(16, 9, 4, 93)
    bn.mu[3, 1] = np.nan
    bn.dn[5, 0] = -1.0
    gn = _gpu(bn, torch.float64, 80, 1e-12, vjp=False)
    assert gn["status"][3] == N.ST_NONFINITE and gn["status"][5] == N.ST_NONFINITE
    assert np.all(gn["status"][[i for i in range(16) if i not in (3, 5)]] == N.ST_CONVERGED)
    z = lambda k, dt=torch.float64: torch.zeros(k, dtype=dt, device="cuda")
    bad = solver.Batch.uniform(4, 9, 10, torch.float64)      # rows not a multiple of 3
    s = bad.sizes()
    with pytest.raises(N.CsError) as e:
        k = s["aref"] // 3
        solver.forward_ell(bad, z(s["M"]), z(s["J"]), z(s["a0"]), z(s["aref"]), z(k), z(k), z(k))
    assert e.value.code == N.CS_EINVAL
    big = solver.Batch.uniform(2, 36, 6, torch.float64)
    s = big.sizes()
    with pytest.raises(N.CsError) as e:
        solver.forward_ell(big, z(s["M"]), z(s["J"]), z(s["a0"]), z(s["aref"]), z(4), z(4), z(4))
    assert e.value.code == N.CS_EUNSUPPORTED
