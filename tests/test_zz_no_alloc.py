"""cs_unrolled_vjp_static -- the unrolled VJP with the library's static tape
(no device allocation) -- against cs_unrolled_vjp with a caller-owned tape,
through the C ABI: two calls in a row, the second with a smaller batch, every
output bitwise equal (same kernels, same inputs)."""
import numpy as np
import pytest
import torch

from paper_2607_24959_amd import _native as N
from paper_2607_24959_amd import solver, synth

pytestmark = pytest.mark.gpu

KEYS = ("M", "J", "a0", "aref", "D", "abar")
OUTS = ("a", "a0", "aref", "J", "D", "M")


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _call(batch, t, K, tol, static):
    vp = solver._vp
    out = {k: torch.full_like(t[k if k != "a" else "a0"], float("nan")) for k in OUTS}
    out["status"] = torch.full((batch.B,), -1, dtype=torch.int32, device="cuda")
    out["iters"] = torch.full((batch.B,), -1, dtype=torch.int32, device="cuda")
    p = N.CsSolverParams(int(K), 0, float(tol))
    args = [vp(t[k]) for k in KEYS] + [vp(out[k]) for k in OUTS]
    stream = solver._stream(torch.device("cuda"))
    if static:
        rc = N.unrolled_vjp_static(batch.desc, p, *args, vp(out["status"]), vp(out["iters"]), stream)
        N.check(rc, "cs_unrolled_vjp_static")
    else:
        tape = torch.empty(max(batch.tape_bytes(K), 1), dtype=torch.uint8, device="cuda")
        rc = N.unrolled_vjp(batch.desc, p, *args, vp(tape), tape.numel(), vp(out["status"]),
                            vp(out["iters"]), stream)
        N.check(rc, "cs_unrolled_vjp")
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_static_tape_matches_caller_tape_twice(dtype):
    _needs_gpu()
    npd = np.float32 if dtype == torch.float32 else np.float64
    # first the benchmark shape at K = 10 (a 36.9 MB FP32 tape), then a
    # smaller batch (the array keeps the first call's contents)
    for B, n, nc, K, path in ((4096, 9, 16, 10, N.PATH_AUTO), (300, 6, 4, 5, N.PATH_TEAM)):
        if dtype == torch.float64 and B == 4096:
            B, n, nc, K = 1024, 6, 4, 10
        hb = synth.uniform_batch(B, n, nc, 20260801 + B).astype(npd)
        batch = solver.Batch.uniform(B, n, 4 * nc, dtype, path=path)
        assert batch.tape_bytes(K) <= N.STATIC_TAPE_BYTES
        t = {k: torch.from_numpy(np.ascontiguousarray(getattr(hb, k))).cuda() for k in KEYS}
        ref = _call(batch, t, K, 1e-5, static=False)
        got = _call(batch, t, K, 1e-5, static=True)
        print(str(dtype), B, n, nc, K, "iters mean", float(ref["iters"].float().mean()))
        for k in OUTS + ("status", "iters"):
            assert torch.equal(got[k], ref[k]), (str(dtype), B, k)
        assert torch.all(torch.isfinite(got["a"]))
