"""The plain unrolled-AD baseline (PyTorch autograd through the K-step solve)
against the oracle's hand-derived unrolled-trace VJP.

The two are independent: one differentiates the batched tensor program by
torch.autograd, the other reverses a recorded trace with adjoints written out
by hand (Sec. III-B steps, eq. 10 line search).  They differentiate the same
function, so on the same inputs they agree to FP64 rounding, and take the same
number of steps.  M-bar is compared symmetrised: M enters the solve through
quadratic forms whose value is the same for M and M^T, so the two programs may
attribute a term to (j, l) or (l, j).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2607_24959_amd import ad_unrolled, synth


@pytest.mark.parametrize("K", [1, 3, 10])
def test_ad_baseline_equals_oracle_unrolled(K):
    B, n, nc = 12, 6, 4
    m = 4 * nc
    hb = synth.uniform_batch(B, n, nc, 20260724 + K)
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(hb, k))).double()
         for k in ("M", "J", "a0", "aref", "D", "abar")}
    out = ad_unrolled.vjp(t["M"], t["J"].reshape(B, m, n), t["a0"], t["aref"], t["D"], t["abar"],
                          K=K, tol=1e-10)
    for i in range(B):
        o = oracle.unrolled_vjp(hb.M[i], hb.J[i], hb.a0[i], hb.aref[i], hb.D[i], hb.abar[i], K,
                                tol=1e-10)
        assert o["iters"] == int(out["steps"][i])
        for key in ("a", "a0", "aref", "J", "D", "M"):
            g = out[key][i].numpy().reshape(o[key].shape)
            ref = o[key]
            if key == "M":
                g, ref = g + g.T, ref + ref.T
            e = np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-300)
            assert e <= 1e-9, (K, i, key, e)


def test_ad_baseline_line_search_is_exact():
    """The batched piece-Newton search returns the exact minimiser (the
    oracle's sorted-breakpoint scan) and its accepted piece, along descent
    directions (the only ones a Newton step produces)."""
    rng = np.random.default_rng(5)
    for i in range(20):
        d = synth.instance(77, i, 9, 16)
        a = d["a0"] + rng.normal(size=9)
        p = rng.normal(size=9)
        J = d["J"].reshape(64, 9)
        r = J @ a - d["aref"]
        w = d["D"] * (r < 0) * r
        if p @ (d["M"] @ (a - d["a0"]) + J.T @ w) > 0:   # phi'(0) < 0
            p = -p
        alpha, Ap, q = oracle.line_search(d["M"], d["J"], d["a0"], d["aref"], d["D"], a, p)
        Mp = d["M"] @ p
        c0, b0 = p @ Mp, Mp @ (a - d["a0"])
        T = lambda x: torch.as_tensor(np.asarray(x, dtype=np.float64)).reshape(1, -1)
        tt, act = ad_unrolled.line_search(T(r), T(q), T(d["D"]), T([c0])[0], T([b0])[0])
        assert alpha > 0
        assert abs(float(tt[0]) - alpha) <= 1e-12 * max(1.0, abs(alpha))
        assert np.array_equal(act[0].numpy(), Ap)
