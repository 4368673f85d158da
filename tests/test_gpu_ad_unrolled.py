"""GPU: the library's unrolled-trace VJP (through the C ABI) against plain
unrolled AD (PyTorch autograd through the same batched K-step solve), and the
memory growth that makes the implicit VJP worth having.

Both differentiate the executed trace, so they agree to rounding wherever they
take the same trace; M-bar is compared symmetrised (see test_ad_unrolled).
"""
import numpy as np
import pytest
import torch

from paper_2607_24959_amd import ad_unrolled, solver, synth

from gpu_common import KEYS, dev, gpu_unrolled_uniform, np64

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
    """Config: B=256, nv=9, 16 contacts (64 rows), FP32, K=10, tol 1e-5."""
    _needs_gpu()
    hb = synth.uniform_batch(256, 9, 16, 20260725).astype(np.float32)
    g = gpu_unrolled_uniform(hb, torch.float32, 10, 1e-5)
    ad = _ad(hb, torch.float32, 10, 1e-5)
    same = g["iters"] == ad["steps"]
    assert same.mean() >= 0.9
    for key, bar in (("a", 1e-4), ("J", 1e-3), ("a0", 1e-3)):
        x, y = g[key].reshape(hb.B, -1)[same], ad[key].reshape(hb.B, -1)[same]
        e = np.linalg.norm(x - y, axis=1) / np.maximum(np.linalg.norm(y, axis=1), 1e-30)
        assert np.median(e) <= bar, (key, np.median(e))


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
