"""GPU: the library's unrolled-trace VJP (through the C ABI) against plain
unrolled AD (PyTorch autograd through the same batched K-step solve), and the
memory growth that makes the implicit VJP worth having.

Both differentiate the executed trace, so they agree to rounding wherever they
take the same trace; M-bar is compared symmetrised (see test_ad_unrolled).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2607_24959_amd import ad_unrolled, solver, synth

from gpu_common import (KEYS, SOLVE_FACTOR, dev, gpu_unrolled_uniform, np64, oracle_traces,
                        solve_cond_bound, tape_trace_uniform)

pytestmark = pytest.mark.gpu


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _ad(hb, dtype, K, tol):
    t = {k: dev(getattr(hb, k), dtype) for k in KEYS + ("abar",)}
    out = ad_unrolled.vjp(t["M"], t["J"].reshape(hb.B, hb.m, hb.n), t["a0"], t["aref"], t["D"],
                          t["abar"], K=K, tol=tol)
    torch.cuda.synchronize()
    return {k: np64(v) if v.dtype.is_floating_point else v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("K", [1, 4, 10])
def test_unrolled_kernel_equals_plain_ad_fp64(K):
    """Config: B=64, nv=6, 4 contacts (16 rows), FP64, tol 1e-10."""
    _needs_gpu()
    hb = synth.uniform_batch(64, 6, 4, 20260724)
    g = gpu_unrolled_uniform(hb, torch.float64, K, 1e-10)
    ad = _ad(hb, torch.float64, K, 1e-10)
    assert np.array_equal(g["iters"], ad["steps"])
    for key in ("a", "a0", "aref", "J", "D", "M"):
        x = g[key].reshape(hb.B, -1)
        y = ad[key].reshape(hb.B, -1)
        if key == "M":
            x = (x.reshape(-1, 6, 6) + x.reshape(-1, 6, 6).transpose(0, 2, 1)).reshape(hb.B, -1)
            y = (y.reshape(-1, 6, 6) + y.reshape(-1, 6, 6).transpose(0, 2, 1)).reshape(hb.B, -1)
        e = np.linalg.norm(x - y, axis=1) / np.maximum(np.linalg.norm(y, axis=1), 1e-300)
        assert e.max() <= 1e-9, (key, e.max())


def test_unrolled_kernel_close_to_plain_ad_fp32():
    """Config: B=256, nv=9, 16 contacts (64 rows), FP32, K=10, tol 1e-5.  Every
    instance where the kernel's trace (its tape) and plain AD's trace both equal
    the oracle's: within 1e-4 (a) / 1e-3 (gradients) of each other, or within
    twice the solve-conditioning bound each FP32 result is held to."""
    _needs_gpu()
    K = 10
    hb = synth.uniform_batch(256, 9, 16, 20260725)
    h32, h64 = hb.astype(np.float32), hb.rounded(np.float32)
    batch = solver.Batch.uniform(hb.B, hb.n, hb.m, torch.float32)
    t = {k: dev(getattr(h32, k), torch.float32) for k in KEYS + ("abar",)}
    tape = torch.empty(max(batch.tape_bytes(K), 1), dtype=torch.uint8, device="cuda")
    out = solver.unrolled_vjp(batch, *(t[k] for k in KEYS), t["abar"], K=K, tol=1e-5, tape=tape)
    tr = []
    ad = ad_unrolled.vjp(t["M"], t["J"].reshape(hb.B, hb.m, hb.n), t["a0"], t["aref"], t["D"],
                         t["abar"], K=K, tol=1e-5, trace=tr)
    torch.cuda.synchronize()
    A, Ap = tape_trace_uniform(tape.cpu().numpy(), hb.B, hb.n, hb.m, K)
    it = out["iters"].cpu().numpy()
    steps = ad["steps"].cpu().numpy()
    adA = np.stack([x[0].cpu().numpy() for x in tr], 1) if tr else np.zeros((hb.B, 0, hb.m), bool)
    adAp = np.stack([x[1].cpu().numpy() for x in tr], 1) if tr else np.zeros((hb.B, 0, hb.m), bool)
    otr = oracle_traces(h64, K, 1e-5)
    same = np.array([otr[i][0] == it[i] == steps[i] and
                     np.array_equal(otr[i][1], A[i, :it[i]]) and np.array_equal(otr[i][2], Ap[i, :it[i]]) and
                     np.array_equal(adA[i, :it[i]], A[i, :it[i]]) and np.array_equal(adAp[i, :it[i]], Ap[i, :it[i]])
                     for i in range(hb.B)])
    print("traces equal (kernel, plain AD, oracle):", same.mean())
    assert same.mean() >= 0.85
    cb = solve_cond_bound(h64, K, 1e-5)
    for key, bar in (("a", 1e-4), ("J", 1e-3), ("a0", 1e-3)):
        x = np64(out[key]).reshape(hb.B, -1)
        y = np64(ad[key]).reshape(hb.B, -1)
        e = np.linalg.norm(x - y, axis=1) / np.maximum(np.linalg.norm(y, axis=1), 1e-30)
        bound = np.maximum(bar, 2 * SOLVE_FACTOR * cb)
        print(key, "max", e[same].max(), "max err/bound", (e / bound)[same].max())
        bad = np.flatnonzero(same & (e > bound))
        assert bad.size == 0, (key, [(int(i), float(e[i]), float(cb[i])) for i in bad[:5]])


def test_plain_ad_memory_grows_with_K_ift_state_does_not():
    """Config: B=512, nv=9, 16 contacts, FP32: autograd keeps every iteration."""
    _needs_gpu()
    hb = synth.uniform_batch(512, 9, 16, 20260726).astype(np.float32)
    t = {k: dev(getattr(hb, k), torch.float32) for k in KEYS + ("abar",)}
    peaks = {}
    for K in (1, 10):
        ad_unrolled.vjp(t["M"], t["J"].reshape(512, 64, 9), t["a0"], t["aref"], t["D"], t["abar"],
                        K=K, tol=1e-5)
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        ad_unrolled.vjp(t["M"], t["J"].reshape(512, 64, 9), t["a0"], t["aref"], t["D"], t["abar"],
                        K=K, tol=1e-5)
        torch.cuda.synchronize()
        peaks[K] = torch.cuda.max_memory_allocated() - base
    batch = solver.Batch.uniform(512, 9, 64, torch.float32)
    print("plain AD peak bytes", peaks, "IFT state bytes", batch.state_bytes())
    assert peaks[10] > 3 * peaks[1]
    assert peaks[10] > 20 * batch.state_bytes()
