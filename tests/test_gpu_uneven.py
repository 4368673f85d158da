"""Uneven (packed) batches on the GPU.

* the full mixed batch (B=8192, nv in {3,9,18,36,96}, 0..256 contacts, FP32)
  planned into tile classes and solved; a stratified sample of instances is
  checked against the FP64 oracle one by one;
* every kernel family on a mixed batch in FP32 and FP64 against the oracle;
* an instance gives bit-identical results alone and inside the mixed batch;
* a captured HIP graph replays to the eager results, several times, with
  eager work in between.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2607_24959_amd import batching, solver, synth
from paper_2607_24959_amd import _native as N

import gpu_common as G

pytestmark = pytest.mark.gpu

TAU_DEG = 1e-7
KEYS = ("M", "J", "a0", "aref", "D", "abar")


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(pb, dtype):
    return {k: torch.from_numpy(np.ascontiguousarray(getattr(pb, k))).to("cuda", dtype) for k in KEYS}


def _check_sample(pb, p64, sol, grads, idx, max_iter, tol_a, tol_g, dtype_label):
    a = sol.a.double().cpu().numpy()
    st = sol.status.cpu().numpy()
    gg = dict(zip(G.GKEYS, (g.double().cpu().numpy() for g in grads)))
    offs = dict(a0=pb.off_n, aref=pb.off_m, J=pb.off_mn, D=pb.off_m, M=pb.off_nn)
    worst, n_checked, n_deg = [], 0, 0
    for i in idx:
        d = p64.get(i)
        res = oracle.forward(d["M"], d["J"], d["a0"], d["aref"], d["D"], max_iter=max_iter, tol=1e-11)
        ao = res["a"]
        if d["m"]:
            r = d["J"] @ ao - d["aref"]
            scale = np.abs(d["aref"]) + np.abs(d["J"]) @ np.abs(ao) + 1e-300
            if (np.abs(r) / scale).min() < TAU_DEG:
                n_deg += 1
                continue
        sl = slice(pb.off_n[i], pb.off_n[i + 1])
        ea = np.linalg.norm(a[sl] - ao) / max(np.linalg.norm(ao), 1e-30)
        assert ea <= tol_a, (dtype_label, i, int(pb.nv[i]), int(pb.nrows[i]), ea)
        if res["status"] != oracle.ST_CONVERGED or st[i] & 1 == 0:
            continue
        og = oracle.ift_vjp(d["M"], d["J"], d["a0"], d["aref"], d["D"], ao, d["abar"],
                            active=res["active"])
        for k in G.GKEYS:
            s2 = slice(offs[k][i], offs[k][i + 1])
            ref = og[k].ravel()
            e = np.linalg.norm(gg[k][s2] - ref) / max(np.linalg.norm(ref), 1e-30)
            worst.append((e, i, k, int(pb.nv[i]), int(pb.nrows[i])))
        n_checked += 1
    worst.sort(reverse=True)
    print(dtype_label, "checked", n_checked, "degenerate", n_deg, "worst", worst[:3])
    bad = [w for w in worst if w[0] > tol_g]
    return n_checked, bad, worst


def test_full_uneven_batch_planned_fp32():
    """B=8192, nv in {3,9,18,36,96}, nc ~ U{0..256}: sampled parity at convergence."""
    _needs_gpu()
    pb = synth.uneven_batch(8192, (3, 9, 18, 36, 96), 256, seed=synth.SEED_BASE + 2)
    p32, p64 = pb.astype(np.float32), pb.rounded(np.float32)
    batch = solver.Batch.packed_from(pb.nv, pb.nrows, torch.float32)
    plan = batching.Plan(batch)
    print(plan.summary())
    t = _dev(p32, torch.float32)
    sol = plan.forward(t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=60, tol=1e-5)
    grads = plan.ift_vjp(sol, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"])
    torch.cuda.synchronize()
    st = sol.status.cpu().numpy()
    assert np.all(st & (N.ST_NONFINITE | N.ST_NOTSPD) == 0)
    # stratified sample: 24 instances of every nv
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.choice(np.flatnonzero(pb.nv == n), 24, replace=False)
                          for n in (3, 9, 18, 36, 96)])
    n_checked, bad, worst = _check_sample(pb, p64, sol, grads, idx, 60, 1e-4, 1e-3, "fp32")
    assert n_checked >= 90
    assert len(bad) <= max(1, n_checked // 20), bad
    assert worst[0][0] <= 1e-2


@pytest.mark.parametrize("path", [N.PATH_TEAM, N.PATH_CHUNK, N.PATH_AUTO])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_families_on_mixed_batch(path, dtype):
    _needs_gpu()
    pb = synth.uneven_batch(60, (3, 9, 18, 36, 96), 48, seed=99)
    npd = np.float32 if dtype == torch.float32 else np.float64
    px = pb.astype(npd)
    p64 = px.astype(np.float64)
    batch = solver.Batch.packed_from(pb.nv, pb.nrows, dtype, path=path)
    t = _dev(px, dtype)
    sol = solver.forward(batch, *(t[k] for k in KEYS[:5]), max_iter=60,
                         tol=1e-5 if dtype == torch.float32 else 1e-12)
    grads = solver.ift_vjp(batch, sol, *(t[k] for k in KEYS[:5]), t["abar"])
    torch.cuda.synchronize()
    tol_a, tol_g = (1e-4, 1e-3) if dtype == torch.float32 else (1e-10, 1e-8)
    n_checked, bad, worst = _check_sample(pb, p64, sol, grads, range(pb.B), 60, tol_a, tol_g,
                                          f"path{path} {dtype}")
    assert n_checked >= 50
    if dtype == torch.float64:
        assert not bad, bad
    else:
        assert len(bad) <= 3, bad


def test_alone_equals_in_mix_bitwise():
    _needs_gpu()
    pb = synth.uneven_batch(300, (3, 9, 18, 36, 96), 64, seed=123)
    p32 = pb.astype(np.float32)
    batch = solver.Batch.packed_from(pb.nv, pb.nrows, torch.float32)
    plan = batching.Plan(batch)
    t = _dev(p32, torch.float32)
    sol = plan.forward(t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=30, tol=1e-5)
    grads = plan.ift_vjp(sol, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"])
    torch.cuda.synchronize()
    a_mix = sol.a.cpu().numpy()
    j_mix = grads[2].cpu().numpy()
    for i in (0, 7, 42, 101, 299):
        d = p32.get(i)
        one = synth.pack([dict(n=d["n"], **{k: d[k] for k in ("M", "J", "a0", "aref", "D", "abar")})])
        one32 = one.astype(np.float32)
        b1 = solver.Batch.packed_from(one.nv, one.nrows, torch.float32)
        p1 = batching.Plan(b1)
        t1 = _dev(one32, torch.float32)
        s1 = p1.forward(t1["M"], t1["J"], t1["a0"], t1["aref"], t1["D"], max_iter=30, tol=1e-5)
        g1 = p1.ift_vjp(s1, t1["M"], t1["J"], t1["a0"], t1["aref"], t1["D"], t1["abar"])
        torch.cuda.synchronize()
        assert np.array_equal(s1.a.cpu().numpy(), a_mix[pb.off_n[i]:pb.off_n[i + 1]]), i
        assert np.array_equal(g1[2].cpu().numpy(), j_mix[pb.off_mn[i]:pb.off_mn[i + 1]]), i


def test_graph_replay_matches_eager():
    _needs_gpu()
    pb = synth.uneven_batch(512, (3, 9, 18, 36, 96), 128, seed=321)
    p32 = pb.astype(np.float32)
    batch = solver.Batch.packed_from(pb.nv, pb.nrows, torch.float32)
    plan = batching.Plan(batch)
    t = _dev(p32, torch.float32)
    ref = plan.forward(t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=10, tol=1e-5)
    gref = plan.ift_vjp(ref, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"])
    torch.cuda.synchronize()
    a_ref, j_ref = ref.a.clone(), gref[2].clone()
    sol, grads = plan.capture(t, max_iter=10, tol=1e-5)
    for rep in range(3):
        sol.a.zero_()
        grads[2].zero_()
        plan.graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(sol.a, a_ref), rep
        assert torch.equal(grads[2], j_ref), rep
        # eager work between replays
        plan.forward(t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=3, tol=1e-5)
        torch.cuda.synchronize()


def test_wave_family_mixed_fp32():
    """One-wave family (J resident in LDS): n in {3, 9, 18, 31}, 0..256 contacts."""
    _needs_gpu()
    pb = synth.uneven_batch(96, (3, 9, 18, 31), 256, seed=77)
    p32 = pb.astype(np.float32)
    p64 = pb.rounded(np.float32)
    batch = solver.Batch.packed_from(pb.nv, pb.nrows, torch.float32, path=N.PATH_WAVE)
    t = _dev(p32, torch.float32)
    sol = solver.forward(batch, *(t[k] for k in KEYS[:5]), max_iter=60, tol=1e-5)
    grads = solver.ift_vjp(batch, sol, *(t[k] for k in KEYS[:5]), t["abar"])
    torch.cuda.synchronize()
    assert np.all(sol.status.cpu().numpy() & (N.ST_NONFINITE | N.ST_NOTSPD) == 0)
    n_checked, bad, worst = _check_sample(pb, p64, sol, grads, range(pb.B), 60, 1e-4, 1e-3, "wave fp32")
    assert n_checked >= 70
    assert len(bad) <= 4, bad
    # the same instances on the chunked family agree to FP32 rounding
    b2 = solver.Batch.packed_from(pb.nv, pb.nrows, torch.float32, path=N.PATH_CHUNK)
    s2 = solver.forward(b2, *(t[k] for k in KEYS[:5]), max_iter=60, tol=1e-5)
    torch.cuda.synchronize()
    conv = (sol.status.cpu().numpy() & 1) & (s2.status.cpu().numpy() & 1)
    a1, a2 = sol.a.cpu().numpy(), s2.a.cpu().numpy()
    errs = [np.linalg.norm(a1[pb.off_n[i]:pb.off_n[i + 1]] - a2[pb.off_n[i]:pb.off_n[i + 1]]) /
            max(np.linalg.norm(a2[pb.off_n[i]:pb.off_n[i + 1]]), 1e-30) for i in range(pb.B) if conv[i]]
    assert np.median(errs) <= 1e-5


def test_wave_family_size_boundaries_fp32():
    """One-wave family at the edges of its compile-time sizes: n in {1, 2, 15,
    16, 17, 20, 21, 23, 24, 25, 28, 29, 30, 31} (Cholesky column counts 16 / 20
    / 24 / 28 / 32, padded widths 16 / 32) with 0, 1, 16, 17 and 256 contacts (0, 4, 64, 68, 1024 rows:
    empty, one K-step, exactly one and just over one row group, the maximum)."""
    _needs_gpu()
    shapes = [(n, nc) for n in (1, 2, 15, 16, 17, 20, 21, 23, 24, 25, 28, 29, 30, 31)
              for nc in (0, 1, 16, 17, 256)]
    pb = synth.pack([synth.instance(4242, i, n, nc) for i, (n, nc) in enumerate(shapes)])
    p32, p64 = pb.astype(np.float32), pb.rounded(np.float32)
    batch = solver.Batch.packed_from(pb.nv, pb.nrows, torch.float32, path=N.PATH_WAVE)
    t = _dev(p32, torch.float32)
    sol = solver.forward(batch, *(t[k] for k in KEYS[:5]), max_iter=60, tol=1e-5)
    grads = solver.ift_vjp(batch, sol, *(t[k] for k in KEYS[:5]), t["abar"])
    torch.cuda.synchronize()
    assert np.all(sol.status.cpu().numpy() & (N.ST_NONFINITE | N.ST_NOTSPD) == 0)
    n_checked, bad, worst = _check_sample(pb, p64, sol, grads, range(pb.B), 60, 1e-4, 1e-3,
                                          "wave boundaries fp32")
    assert n_checked >= 0.8 * pb.B
    assert len(bad) <= 2, bad


def test_wave_family_rejects_fp64_and_large_n():
    _needs_gpu()
    for dtype, n, m in ((torch.float64, 9, 8), (torch.float32, 36, 8), (torch.float32, 9, 1028)):
        batch = solver.Batch.uniform(4, n, m, dtype, path=N.PATH_WAVE)
        z = lambda k: torch.zeros(k, dtype=dtype, device="cuda")
        s = batch.sizes()
        with pytest.raises(N.CsError) as e:
            solver.forward(batch, z(s["M"]), z(s["J"]), z(s["a0"]), z(s["aref"]), z(s["D"]))
        assert e.value.code == N.CS_EUNSUPPORTED
