"""Equality rows as pairs of one-sided rows (paper_2607_24959_amd/rows.py),
checked with the oracle against the closed form of the equality-only problem
and its derivative:

  minimise 1/2 (a - a0)^T M (a - a0) + 1/2 sum_e D_e (J_e a - aref_e)^2
  =>  a* = (M + Je^T De Je)^{-1} (M a0 + Je^T De arefe),

differentiated by torch autograd in FP64 (an independent derivation); and,
with contact rows present, the expanded problem's solution and folded VJP
against central differences of the oracle."""
import numpy as np
import torch

import oracle
from paper_2607_24959_amd import rows, synth


def _closed(M, Je, a0, arefe, De):
    H = M + Je.T @ (De[:, None] * Je)
    return torch.linalg.solve(H, M @ a0 + Je.T @ (De * arefe))


def test_equality_only_matches_closed_form_and_its_gradient():
    rng = np.random.default_rng(1)
    b = synth.uniform_batch(8, 6, 0, 17)
    for i in range(8):
        k = 3
        Je = rng.standard_normal((k, 6))
        arefe = rng.standard_normal(k) * 10
        De = 10 ** rng.uniform(0, 2, k)
        t = lambda x: torch.tensor(x, dtype=torch.float64)
        J2, aref2, D2 = rows.with_equality_rows(t(np.zeros((1, 0, 6))), t(np.zeros((1, 0))),
                                                t(np.zeros((1, 0))), t(Je[None]), t(arefe[None]),
                                                t(De[None]))
        J2, aref2, D2 = J2[0].numpy(), aref2[0].numpy(), D2[0].numpy()
        r = oracle.forward(b.M[i], J2, b.a0[i], aref2, D2, max_iter=40, tol=1e-13)
        assert r["status"] == oracle.ST_CONVERGED
        ref = _closed(t(b.M[i]), t(Je), t(b.a0[i]), t(arefe), t(De)).numpy()
        assert np.abs(r["a"] - ref).max() <= 1e-11 * np.abs(ref).max()
        # gradient of abar . a* w.r.t. (Je, arefe, De) through the pairs
        g = oracle.ift_vjp(b.M[i], J2, b.a0[i], aref2, D2, r["a"], b.abar[i], active=r["active"])
        _, (Jeb, arb, Deb) = rows.fold_equality_grads(t(g["J"]), t(g["aref"]), t(g["D"]), 0, k)
        Jt, at, Dt = (t(x).requires_grad_(True) for x in (Je, arefe, De))
        (t(b.abar[i]) @ _closed(t(b.M[i]), Jt, t(b.a0[i]), at, Dt)).backward()
        for got, want in ((Jeb, Jt.grad), (arb, at.grad), (Deb, Dt.grad)):
            assert torch.allclose(got, want, rtol=1e-9, atol=1e-12 * want.abs().max().item())


def test_equality_with_contacts_against_fd():
    rng = np.random.default_rng(2)
    b = synth.uniform_batch(4, 6, 4, 23)
    t = lambda x: torch.tensor(x, dtype=torch.float64)
    for i in range(4):
        k = 2
        Je = rng.standard_normal((k, 6))
        arefe = rng.standard_normal(k) * 10
        De = 10 ** rng.uniform(0, 2, k)

        def solve(Je_, arefe_, De_):
            J2, aref2, D2 = rows.with_equality_rows(t(b.J[i][None]), t(b.aref[i][None]),
                                                    t(b.D[i][None]), t(Je_[None]), t(arefe_[None]),
                                                    t(De_[None]))
            return J2[0].numpy(), aref2[0].numpy(), D2[0].numpy()

        J2, aref2, D2 = solve(Je, arefe, De)
        r = oracle.forward(b.M[i], J2, b.a0[i], aref2, D2, max_iter=60, tol=1e-13)
        assert r["status"] == oracle.ST_CONVERGED
        g = oracle.ift_vjp(b.M[i], J2, b.a0[i], aref2, D2, r["a"], b.abar[i], active=r["active"])
        _, (Jeb, arb, Deb) = rows.fold_equality_grads(t(g["J"]), t(g["aref"]), t(g["D"]), b.m, k)
        for X, G in ((Je, Jeb), (arefe, arb), (De, Deb)):
            dX = rng.standard_normal(X.shape)
            eps = 1e-6 * max(1.0, np.abs(X).max())
            sols = []
            for sg in (1, -1):
                Xp = X + sg * eps * dX
                args = [Je, arefe, De]
                args[[id(Je), id(arefe), id(De)].index(id(X))] = Xp
                J2p, arp, D2p = solve(*args)
                rp = oracle.forward(b.M[i], J2p, b.a0[i], arp, D2p, max_iter=60, tol=1e-13)
                sols.append(rp)
            if not all(np.array_equal(s["active"], r["active"]) for s in sols):
                continue
            fd = b.abar[i] @ (sols[0]["a"] - sols[1]["a"]) / (2 * eps)
            an = float((G.numpy() * dX).sum())
            assert abs(fd - an) <= 1e-5 * (abs(an) + 1e-6), (i, fd, an)
