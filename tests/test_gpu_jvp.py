"""cs_ift_jvp (forward-mode IFT, eq. 15) through the C ABI against the
oracle's JVP, instance by instance, and the iLQR step Jacobians built from it
against central finite differences of one rollout step."""
import numpy as np
import pytest
import torch

import oracle
from paper_2607_24959_amd import _native as N
from paper_2607_24959_amd import solver, synth
from paper_2607_24959_amd.rollout import make_rollout_problem, step_jacobians

import gpu_common as G

pytestmark = pytest.mark.gpu


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _jvp_case(pb, dtype, k, tol, seed, path=0):
    """Forward + JVP of packed batch pb on the GPU; oracle JVP at the GPU's own
    active sets (the JVP depends on a* only through A*).  Returns per-instance
    relative errors of the k directions."""
    npd = np.float32 if dtype == torch.float32 else np.float64
    px = pb.astype(npd)
    p64 = px.astype(np.float64)
    batch = solver.Batch.packed_from(pb.nv, pb.nrows, dtype, path=path)
    t = {key: G.dev(getattr(px, key), dtype) for key in G.KEYS}
    sol = solver.forward(batch, *(t[key] for key in G.KEYS), max_iter=60, tol=tol)
    rng = np.random.default_rng(seed)
    d0 = rng.standard_normal(k * int(pb.off_n[-1])).astype(npd)
    dr = rng.standard_normal(k * int(pb.off_m[-1])).astype(npd)
    da = solver.ift_jvp(batch, sol, t["M"], t["J"], t["D"], k, G.dev(d0, dtype), G.dev(dr, dtype))
    torch.cuda.synchronize()
    act = batch.active_sets(sol)
    P = oracle.Packed(pb.nv, pb.nrows, p64.M, p64.J, p64.a0, p64.aref, p64.D, p64.abar)
    ref = P.ift_jvp(act, k, d0.astype(np.float64), dr.astype(np.float64))
    got = G.np64(da)
    off = k * pb.off_n
    return G.seg_rel(got, ref, off), sol.status.cpu().numpy()


def test_jvp_fp64_uniform_matches_oracle():
    _needs_gpu()
    b = synth.uniform_batch(64, 6, 4, synth.SEED_BASE)
    pb = synth.pack([dict(n=b.n, M=b.M[i], J=b.J[i], a0=b.a0[i], aref=b.aref[i], D=b.D[i],
                          abar=b.abar[i]) for i in range(b.B)])
    e, st = _jvp_case(pb, torch.float64, 5, 1e-12, 1)
    assert np.all(st & oracle.ST_CONVERGED)
    assert e.max() <= 1e-10, e.max()


@pytest.mark.parametrize("path", [N.PATH_AUTO, N.PATH_TEAM])
def test_jvp_fp32_uneven_matches_oracle(path):
    """FP32, n in {3, 9, 18, 36, 96}, 0..128 contacts, 7 directions: every
    instance within 1e-5 of the oracle at the same active set."""
    _needs_gpu()
    pb = synth.uneven_batch(60, (3, 9, 18, 36, 96), 128, seed=88)
    e, st = _jvp_case(pb, torch.float32, 7, 1e-5, 2, path=path)
    print("FP32 JVP max rel err", e.max())
    assert e.max() <= 1e-5, (e.max(), int(np.argmax(e)))


def test_jvp_edges():
    _needs_gpu()
    b = solver.Batch.uniform(4, 97, 8, torch.float32)
    s = b.sizes()
    z = lambda k: torch.zeros(max(k, 1), device="cuda")
    sol = solver.Solution(a=z(s["a"]), state=torch.zeros(b.state_bytes(), dtype=torch.uint8, device="cuda"),
                          status=torch.zeros(4, dtype=torch.int32, device="cuda"),
                          iters=torch.zeros(4, dtype=torch.int32, device="cuda"))
    with pytest.raises(N.CsError) as e:
        solver.ift_jvp(b, sol, z(s["M"]), z(s["J"]), z(s["D"]), 2, z(2 * s["a0"]), None)
    assert e.value.code == N.CS_EUNSUPPORTED
    # k = 0 is a no-op
    b2 = solver.Batch.uniform(4, 6, 8, torch.float32)
    s2 = b2.sizes()
    out = torch.full((1,), 7.0, device="cuda")
    sol2 = solver.Solution(a=z(s2["a"]), state=torch.zeros(b2.state_bytes(), dtype=torch.uint8, device="cuda"),
                           status=torch.zeros(4, dtype=torch.int32, device="cuda"),
                           iters=torch.zeros(4, dtype=torch.int32, device="cuda"))
    solver.ift_jvp(b2, sol2, z(s2["M"]), z(s2["J"]), z(s2["D"]), 0, None, None, out=out)
    torch.cuda.synchronize()
    assert out.item() == 7.0


def test_ilqr_step_jacobians_match_fd():
    """A_t = dv_{t+1}/dv_t and B_t = dv_{t+1}/dtau_t of one semi-implicit step
    (B=256, nv=18, 32 contacts, FP64) against central differences on instances
    whose active set is the same at every perturbation.  With the active set
    fixed the solution is affine in (a0, aref), so central differences carry no
    truncation error and eps = 1e-3 keeps the solves' rounding negligible
    (B_t = h H^{-1} is small in the stiff directions)."""
    _needs_gpu()
    P = make_rollout_problem(256, 18, 32, 1, seed=20260740)
    M, J, D, pen, v, tau = P["M"], P["J"], P["D"], P["pen"], P["v0"], P["tau"][0]
    Bn, m, n = J.shape
    batch = solver.Batch.uniform(Bn, n, m, torch.float64)
    Minv = torch.linalg.inv(M)
    pen_rows = torch.repeat_interleave(pen, 4, dim=-1)
    h = 0.002

    def step(v, tau):
        a0 = torch.bmm(Minv, tau.unsqueeze(-1)).squeeze(-1)
        aref = -synth.B_DAMP * torch.bmm(J, v.unsqueeze(-1)).squeeze(-1) - synth.K_SPRING * pen_rows
        sol = solver.forward(batch, M, J, a0.contiguous(), aref.contiguous(), D, max_iter=80, tol=1e-13)
        return v + h * sol.a.reshape(Bn, n), sol

    _, sol = step(v, tau)
    A_t, B_t = step_jacobians(M, J, D, sol, batch, h)
    act0 = batch.active_sets(sol).reshape(Bn, m)
    eps = 1e-3
    fdA = torch.zeros_like(A_t)
    fdB = torch.zeros_like(B_t)
    same = np.ones(Bn, bool)
    for j in range(n):
        e = torch.zeros(n, dtype=torch.float64, device="cuda")
        e[j] = eps
        for which, fd in (("v", fdA), ("tau", fdB)):
            vp, sp = step(v + e, tau) if which == "v" else step(v, tau + e)
            vm, sm = step(v - e, tau) if which == "v" else step(v, tau - e)
            fd[:, :, j] = (vp - vm) / (2 * eps)
            same &= np.all(batch.active_sets(sp).reshape(Bn, m) == act0, axis=1)
            same &= np.all(batch.active_sets(sm).reshape(Bn, m) == act0, axis=1)
    torch.cuda.synchronize()
    eA = (torch.linalg.norm(A_t - fdA, dim=(1, 2)) / torch.linalg.norm(fdA, dim=(1, 2))).cpu().numpy()
    eB = (torch.linalg.norm(B_t - fdB, dim=(1, 2)) / torch.linalg.norm(fdB, dim=(1, 2))).cpu().numpy()
    print("iLQR Jacobians vs FD: valid", same.mean(), "A max", eA[same].max(), "B max", eB[same].max())
    assert same.mean() >= 0.9
    assert eA[same].max() <= 1e-6 and eB[same].max() <= 1e-6
