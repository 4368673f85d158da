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

KEYS = ("M", "J", "a0", "aref", "D", "abar")


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(pb, dtype):
    return {k: torch.from_numpy(np.ascontiguousarray(getattr(pb, k))).to("cuda", dtype) for k in KEYS}


def _check_fp64_packed(pb, g, max_iter, label):
    """FP64 results: every instance within 1e-10 (a) and 1e-8 (gradients), same
    status and active set."""
    P = oracle.Packed(pb.nv, pb.nrows, pb.M, pb.J, pb.a0, pb.aref, pb.D, pb.abar)
    fw = P.forward(max_iter=max_iter, tol=1e-11)
    assert np.array_equal(g["status"], fw["status"]), label
    assert np.array_equal(g["active"].astype(bool), fw["active"][:int(pb.off_m[-1])].astype(bool)), label
    ea = G.seg_rel(g["a"], fw["a"], pb.off_n)
    assert ea.max() <= 1e-10, (label, ea.max())
    og = P.ift_vjp(fw["a"], fw["active"])
    for k, off in G.grad_offsets(P).items():
        e = G.seg_rel(g[k], og[k], off)
        assert e.max() <= 1e-8, (label, k, e.max(), int(np.argmax(e)))


def test_full_uneven_batch_planned_fp32():
    """B=8192, nv in {3,9,18,36,96}, nc ~ U{0..256}: planned into tile classes
    and solved; a stratified sample (24 instances of every nv) is checked
    instance by instance against the oracle."""
    _needs_gpu()
    pb = synth.uneven_batch(8192, (3, 9, 18, 36, 96), 256, seed=synth.SEED_BASE + 2)
    g = G.gpu_packed(pb, torch.float32, 60, 1e-5, plan=True)
    assert np.all(g["status"] & (N.ST_NONFINITE | N.ST_NOTSPD) == 0)
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.choice(np.flatnonzero(pb.nv == n), 24, replace=False)
                          for n in (3, 9, 18, 36, 96)])
    sub, gs = G.subset(pb, g, idx)
    G.check_fp32("uneven 8192 sample", G.oracle_packed(sub), gs, max_iter=60)


@pytest.mark.parametrize("path", [N.PATH_TEAM, N.PATH_CHUNK, N.PATH_AUTO])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_families_on_mixed_batch(path, dtype):
    _needs_gpu()
    pb = synth.uneven_batch(60, (3, 9, 18, 36, 96), 48, seed=99)
    if dtype == torch.float64:
        g = G.gpu_packed(pb, dtype, 60, 1e-12, path=path)
        _check_fp64_packed(pb, g, 60, f"path{path} fp64")
    else:
        g = G.gpu_packed(pb, dtype, 60, 1e-5, path=path)
        G.check_fp32(f"mixed path{path}", G.oracle_packed(pb), g, max_iter=60)


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


@pytest.mark.parametrize("lanes", [1, 2])
def test_graph_replay_matches_eager(lanes):
    """The captured graph (classes on one stream, or dealt to two concurrent
    streams) replays to the eager results bitwise, several times, with eager
    work in between."""
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
    sol, grads = plan.capture(t, max_iter=10, tol=1e-5, lanes=lanes)
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
    g = G.gpu_packed(pb, torch.float32, 60, 1e-5, path=N.PATH_WAVE)
    assert np.all(g["status"] & (N.ST_NONFINITE | N.ST_NOTSPD) == 0)
    G.check_fp32("wave mixed", G.oracle_packed(pb), g, max_iter=60)
    # the same instances on the chunked family: both refined to FP32 rounding
    g2 = G.gpu_packed(pb, torch.float32, 60, 1e-5, path=N.PATH_CHUNK, vjp=False)
    e = G.seg_rel(g["a"], g2["a"], pb.off_n)
    assert e.max() <= 1e-6, e.max()


def test_wave_family_size_boundaries_fp32():
    """One-wave family at the edges of its compile-time sizes: n in {1, 2, 15,
    16, 17, 20, 21, 23, 24, 25, 28, 29, 30, 31} (Cholesky column counts 16 / 20
    / 24 / 28 / 32, padded widths 16 / 32) with 0, 1, 16, 17 and 256 contacts (0, 4, 64, 68, 1024 rows:
    empty, one K-step, exactly one and just over one row group, the maximum)."""
    _needs_gpu()
    shapes = [(n, nc) for n in (1, 2, 15, 16, 17, 20, 21, 23, 24, 25, 28, 29, 30, 31)
              for nc in (0, 1, 16, 17, 256)]
    pb = synth.pack([synth.instance(4242, i, n, nc) for i, (n, nc) in enumerate(shapes)])
    g = G.gpu_packed(pb, torch.float32, 60, 1e-5, path=N.PATH_WAVE)
    assert np.all(g["status"] & (N.ST_NONFINITE | N.ST_NOTSPD) == 0)
    G.check_fp32("wave boundaries", G.oracle_packed(pb), g, max_iter=60)


def test_wave_family_rejects_fp64_and_large_n():
    _needs_gpu()
    for dtype, n, m in ((torch.float64, 9, 8), (torch.float32, 36, 8), (torch.float32, 9, 1028)):
        batch = solver.Batch.uniform(4, n, m, dtype, path=N.PATH_WAVE)
        z = lambda k: torch.zeros(k, dtype=dtype, device="cuda")
        s = batch.sizes()
        with pytest.raises(N.CsError) as e:
            solver.forward(batch, z(s["M"]), z(s["J"]), z(s["a0"]), z(s["aref"]), z(s["D"]))
        assert e.value.code == N.CS_EUNSUPPORTED
