"""Equality rows (as pairs of one-sided rows) through the GPU solver and its
IFT VJP, against the oracle on the same expanded rows and, for equality rows
alone, the closed form (M + Je^T De Je)^{-1} (M a0 + Je^T De arefe)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2607_24959_amd import rows, solver, synth

pytestmark = pytest.mark.gpu


def test_equality_rows_fp64_against_oracle_and_closed_form():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(3)
    B, n, nc, k = 64, 6, 4, 3
    b = synth.uniform_batch(B, n, nc, 29)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda", torch.float64)
    Je = rng.standard_normal((B, k, n))
    arefe = rng.standard_normal((B, k)) * 10
    De = 10 ** rng.uniform(0, 2, (B, k))
    for with_contacts in (False, True):
        J = dev(b.J if with_contacts else np.zeros((B, 0, n)))
        aref = dev(b.aref if with_contacts else np.zeros((B, 0)))
        D = dev(b.D if with_contacts else np.zeros((B, 0)))
        J2, aref2, D2 = rows.with_equality_rows(J, aref, D, dev(Je), dev(arefe), dev(De))
        m2 = J2.shape[1]
        batch = solver.Batch.uniform(B, n, m2, torch.float64)
        M, a0, abar = dev(b.M), dev(b.a0), dev(b.abar)
        sol = solver.forward(batch, M, J2, a0, aref2, D2, max_iter=60, tol=1e-12)
        g = solver.ift_vjp(batch, sol, M, J2, a0, aref2, D2, abar)
        torch.cuda.synchronize()
        a = sol.a.cpu().numpy()
        Jn, arn, Dn = J2.cpu().numpy(), aref2.cpu().numpy(), D2.cpu().numpy()
        for i in range(B):
            o = oracle.forward(b.M[i], Jn[i], b.a0[i], arn[i], Dn[i], max_iter=60, tol=1e-12)
            assert np.abs(a[i] - o["a"]).max() <= 1e-10 * np.abs(o["a"]).max(), i
            og = oracle.ift_vjp(b.M[i], Jn[i], b.a0[i], arn[i], Dn[i], o["a"], b.abar[i],
                                active=o["active"])
            got = g[2].cpu().numpy()[i]
            assert np.abs(got - og["J"]).max() <= 1e-8 * np.abs(og["J"]).max(), i
            if not with_contacts:
                H = b.M[i] + Je[i].T @ (De[i][:, None] * Je[i])
                ref = np.linalg.solve(H, b.M[i] @ b.a0[i] + Je[i].T @ (De[i] * arefe[i]))
                assert np.abs(a[i] - ref).max() <= 1e-10 * np.abs(ref).max(), i
