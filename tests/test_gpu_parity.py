"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (per instance, norm-wise relative error):
  FP64 runs: a <= 1e-10, gradients <= 1e-9 (both sides do the same method in
  the same precision; only summation order and QR vs Cholesky differ).
  FP32 runs: a <= 1e-4, gradients <= 1e-3 against the oracle run on the
  FP32-rounded inputs.  Active sets must match except on instances whose
  solution has a row within tau = 1e-7 (relative) of the cone boundary
  ("degenerate"); that fraction is checked to stay below 1 %.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2607_24959_amd import solver, synth
from paper_2607_24959_amd import _native as N

import gpu_common as G

pytestmark = pytest.mark.gpu

TAU_DEG = 1e-7


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check_fp64(g, o, b, label):
    B = b.B
    assert np.array_equal(g["status"], o["status"]), label
    assert np.array_equal(g["iters"], o["iters"]), label
    assert np.array_equal(g["active"], o["active"]), label
    ea = G.rel_rows(g["a"], o["a"], B)
    assert ea.max() <= 1e-10, (label, ea.max())
    conv = o["status"] == oracle.ST_CONVERGED
    for k in G.GKEYS:
        e = G.rel_rows(g[k], o[k], B)[conv]
        assert e.max() <= 1e-9, (label, k, e.max())


@pytest.mark.parametrize("path", [N.PATH_TEAM, N.PATH_SMALL])
def test_fp64_b64_n6_nc4(path):
    """Plain method in FP64: B=64, nv=6, 4 contacts (16 rows), K=10, tol 1e-10."""
    _needs_gpu()
    b = synth.uniform_batch(64, 6, 4, synth.SEED_BASE + 0)
    g = G.gpu_uniform(b, torch.float64, 10, 1e-10, path=path)
    o = G.oracle_uniform(b, 10, 1e-10)
    _check_fp64(g, o, b, f"path{path}")


@pytest.mark.parametrize("K", [0, 1, 3, 10])
@pytest.mark.parametrize("path", [N.PATH_TEAM, N.PATH_SMALL])
def test_fp64_unrolled(K, path):
    _needs_gpu()
    b = synth.uniform_batch(64, 6, 4, synth.SEED_BASE + 0)
    gu = G.gpu_unrolled_uniform(b, torch.float64, K, 1e-10, path=path)
    ou = G.oracle_unrolled_uniform(b, K, 1e-10)
    assert np.array_equal(gu["status"], ou["status"])
    assert np.array_equal(gu["iters"], ou["iters"])
    assert G.rel_rows(gu["a"], ou["a"], b.B).max() <= 1e-10
    for k in G.GKEYS:
        assert G.rel_rows(gu[k], ou[k], b.B).max() <= 1e-8, k


def _fp32_report(g, o, b64, label, conv_only=True):
    B = b64.B
    mg = G.margins(b64, o["a"]).min(axis=1)
    deg = mg < TAU_DEG
    act_eq = np.all(g["active"] == o["active"], axis=1)
    ea = G.rel_rows(g["a"], o["a"], B)
    info = dict(label=label, degenerate=float(deg.mean()), act_mismatch_nondeg=int((~act_eq & ~deg).sum()),
                a_max=float(ea.max()), a_p99=float(np.percentile(ea, 99)))
    print(info)
    return deg, act_eq, ea


@pytest.mark.parametrize("path", [N.PATH_TEAM, N.PATH_SMALL])
def test_fp32_b4096_n9_nc16_converged(path):
    """Uniform FP32 batch B=4096, nv=9, 16 contacts, solved to convergence."""
    _needs_gpu()
    b = synth.uniform_batch(4096, 9, 16, synth.SEED_BASE + 1)
    b32, b64 = b.astype(np.float32), b.rounded(np.float32)
    g = G.gpu_uniform(b32, torch.float32, 50, 1e-5, path=path)
    o = G.oracle_uniform(b64, 50, 1e-10)
    deg, act_eq, ea = _fp32_report(g, o, b64, f"path{path}")
    assert deg.mean() < 0.01
    assert np.all(act_eq | deg)
    assert np.all(g["status"] == oracle.ST_CONVERGED)
    assert ea.max() <= 1e-4
    ok = (o["status"] == oracle.ST_CONVERGED) & act_eq & ~deg
    for k in G.GKEYS:
        e = G.rel_rows(g[k], o[k], b64.B)[ok]
        # D-bar = -A r* sigma inherits the relative error of r* = J a* - aref,
        # which is small for stiff rows; allow 0.1 % of instances past 1e-3
        assert np.mean(e > 1e-3) <= 1e-3, (k, np.sort(e)[-5:])
        assert np.percentile(e, 99) <= 5e-4, k


@pytest.mark.parametrize("K", [1, 5, 10])
@pytest.mark.parametrize("path", [N.PATH_TEAM, N.PATH_SMALL])
def test_fp32_unrolled(K, path):
    """Unrolled FP32 trace gradients: the trace derivative is sensitive to
    rounding along a non-converged path, so agreement is checked by quantiles."""
    _needs_gpu()
    b = synth.uniform_batch(1024, 9, 16, synth.SEED_BASE + 1)
    b32, b64 = b.astype(np.float32), b.rounded(np.float32)
    gu = G.gpu_unrolled_uniform(b32, torch.float32, K, 1e-5, path=path)
    ou = G.oracle_unrolled_uniform(b64, K, 1e-10)
    ea = G.rel_rows(gu["a"], ou["a"], b.B)
    assert np.mean(ea <= 1e-4) >= 0.99
    same = gu["iters"] == ou["iters"]
    for k in G.GKEYS:
        e = G.rel_rows(gu[k], ou[k], b.B)[same]
        print(K, path, k, np.median(e), np.percentile(e, 90))
        assert np.median(e) <= 1e-3, k


def test_fp32_b4096_n9_nc16_cap10():
    """The benchmarked launch: same batch, K=10 cap (most instances stop at the cap)."""
    _needs_gpu()
    b = synth.uniform_batch(4096, 9, 16, synth.SEED_BASE + 1)
    b32, b64 = b.astype(np.float32), b.rounded(np.float32)
    g = G.gpu_uniform(b32, torch.float32, 10, 1e-5)
    o = G.oracle_uniform(b64, 10, 1e-10)
    deg, act_eq, ea = _fp32_report(g, o, b64, "cap10")
    # the K=10 iterate is path dependent: require agreement on 99.5 % of instances
    assert np.mean(ea <= 1e-4) >= 0.995
    both = (g["status"] == oracle.ST_CONVERGED) & (o["status"] == oracle.ST_CONVERGED) & act_eq & ~deg
    for k in G.GKEYS:
        e = G.rel_rows(g[k], o[k], b64.B)[both]
        assert np.mean(e > 1e-3) <= 1e-3, k


@pytest.mark.parametrize("B", [1, 15, 17, 37])
def test_small_kernel_ragged_batches(B):
    """Batches that do not fill the last group of 16 lanes / workgroup of 16 instances."""
    _needs_gpu()
    b = synth.uniform_batch(B, 9, 16, 777 + B)
    b32, b64 = b.astype(np.float32), b.rounded(np.float32)
    g = G.gpu_uniform(b32, torch.float32, 50, 1e-5, path=N.PATH_SMALL)
    o = G.oracle_uniform(b64, 50, 1e-10)
    assert G.rel_rows(g["a"], o["a"], B).max() <= 1e-4


@pytest.mark.parametrize("n,nc", [(1, 1), (3, 0), (3, 2), (6, 16), (12, 16), (12, 5)])
@pytest.mark.parametrize("path", [N.PATH_TEAM, N.PATH_AUTO])
def test_shapes_fp32(n, nc, path):
    _needs_gpu()
    b = synth.uniform_batch(48, n, nc, 99 + n * 100 + nc)
    b32, b64 = b.astype(np.float32), b.rounded(np.float32)
    g = G.gpu_uniform(b32, torch.float32, 60, 1e-5, path=path)
    o = G.oracle_uniform(b64, 60, 1e-10)
    mg = G.margins(b64, o["a"]).min(axis=1) if nc else np.ones(b.B)
    ok = mg >= TAU_DEG
    assert G.rel_rows(g["a"], o["a"], b.B)[ok].max() <= 1e-4
    if nc:
        assert np.all(np.all(g["active"] == o["active"], axis=1)[ok])


def test_packed_uneven_fp32_team():
    """Packed batch of mixed shapes (n in {3,9,18,36,96}, 0..64 contacts)."""
    _needs_gpu()
    pb = synth.uneven_batch(40, (3, 9, 18, 36, 96), 64, seed=4242)
    p32 = pb.astype(np.float32)
    p64 = pb.rounded(np.float32)
    batch = solver.Batch.packed_from(pb.nv, pb.nrows, torch.float32)
    t = {k: G.dev(getattr(p32, k), torch.float32) for k in G.KEYS + ("abar",)}
    sol = solver.forward(batch, *(t[k] for k in G.KEYS), max_iter=60, tol=1e-5)
    gr = solver.ift_vjp(batch, sol, *(t[k] for k in G.KEYS), t["abar"])
    torch.cuda.synchronize()
    P = oracle.Packed(pb.nv, pb.nrows, p64.M, p64.J, p64.a0, p64.aref, p64.D, p64.abar)
    fw = P.forward(max_iter=60, tol=1e-10)
    og = P.ift_vjp(fw["a"], fw["active"])
    a = G.np64(sol.a)
    st = sol.status.cpu().numpy()
    gg = dict(zip(G.GKEYS, (G.np64(x) for x in gr)))
    offs = dict(a0=pb.off_n, aref=pb.off_m, J=pb.off_mn, D=pb.off_m, M=pb.off_nn)
    n_checked = 0
    worst = []
    for i in range(pb.B):
        d = p64.get(i)
        sl = slice(pb.off_n[i], pb.off_n[i + 1])
        ai, ao = a[sl], fw["a"][sl]
        r = d["J"] @ ao - d["aref"]
        scale = np.abs(d["aref"]) + np.abs(d["J"]) @ np.abs(ao) + 1e-300
        if d["m"] and (np.abs(r) / scale).min() < TAU_DEG:
            continue
        assert st[i] == oracle.ST_CONVERGED == fw["status"][i]
        assert np.linalg.norm(ai - ao) <= 1e-4 * max(np.linalg.norm(ao), 1e-30), i
        for k in G.GKEYS:
            s2 = slice(offs[k][i], offs[k][i + 1])
            ref = og[k][s2]
            e = np.linalg.norm(gg[k][s2] - ref) / max(np.linalg.norm(ref), 1e-30)
            worst.append((e, i, k, int(pb.nv[i]), int(pb.nrows[i])))
        n_checked += 1
    assert n_checked >= 36
    worst.sort(reverse=True)
    print("largest gradient errors (err, instance, grad, n, m):", worst[:5])
    # FP32 holds a* to one ulp; on large stiff instances the forces D (J a* - aref)
    # and so the gradients inherit that: a few instances may pass 1e-3
    bad = [w for w in worst if w[0] > 1e-3]
    assert len(bad) <= max(1, n_checked // 20), bad
    assert worst[0][0] <= 1e-2, worst[:3]


def test_status_codes_on_gpu():
    _needs_gpu()
    b = synth.uniform_batch(20, 6, 4, 5)
    b.aref[3, 2] = np.nan          # non-finite input
    b.M[7] = -np.eye(6)            # not positive definite
    for path in (N.PATH_TEAM, N.PATH_SMALL):
        g = G.gpu_uniform(b, torch.float64, 10, 1e-10, vjp=False, path=path)
        assert g["status"][3] == N.ST_NONFINITE and np.isnan(g["a"][3]).all()
        assert g["status"][7] == N.ST_NOTSPD and np.isnan(g["a"][7]).all()
        others = [i for i in range(20) if i not in (3, 7)]
        assert np.all(np.isfinite(g["a"][others]))


def test_order_permutation_and_determinism():
    """Results do not depend on processing order, and repeat bitwise."""
    _needs_gpu()
    b = synth.uniform_batch(300, 9, 16, 8)
    b32 = b.astype(np.float32)
    perm = np.random.default_rng(0).permutation(300)
    for path in (N.PATH_TEAM, N.PATH_SMALL):
        g1 = G.gpu_uniform(b32, torch.float32, 30, 1e-5, path=path)
        g2 = G.gpu_uniform(b32, torch.float32, 30, 1e-5, path=path)
        g3 = G.gpu_uniform(b32, torch.float32, 30, 1e-5, order=perm, path=path)
        for k in ("a",) + G.GKEYS:
            assert np.array_equal(g1[k], g2[k]), k
            assert np.array_equal(g1[k], g3[k]), k
