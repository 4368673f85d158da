"""Pins of the oracle's nonlinear conjugate-gradient forward (Sec. III-B: a
second iterative solver for the same unique minimiser):

* instances built backwards from a chosen minimiser with every row active
  there: CG ends at that minimiser with every row active;
* no contact rows: the minimiser is a0, reached before any step;
* random instances of the benchmark's shape: the CG result satisfies the
  stationarity condition F(a) = 0 of eq. 6 (formed here in numpy), and agrees
  with the separately pinned Newton oracle on a and the active set;
* the packed-batch entry equals the single-instance one.
"""
import numpy as np

import oracle
from paper_2607_24959_amd import synth


def _stationarity(M, J, a0, aref, D, a):
    r = J @ a - aref
    return M @ (a - a0) + J.T @ (D * (r < 0) * r)


def test_quadratic_with_known_minimiser():
    """Instances built backwards from a chosen minimiser a* with every row
    active there (r* < 0): a0 = a* + M^{-1} J^T (D o r*), aref = J a* - r*.
    The objective near a* is one quadratic, a* is its closed-form minimiser,
    and CG must end there with every row active."""
    rng = np.random.default_rng(5)
    for n, m in ((3, 8), (6, 16), (9, 36), (12, 48), (18, 72)):
        A = rng.standard_normal((n, n))
        M = A @ A.T + n * np.eye(n)
        J = rng.standard_normal((m, n))
        D = 10 ** rng.uniform(-1, 2, m)
        a_star = rng.standard_normal(n)
        r_star = -(1 + rng.random(m))
        a0 = a_star + np.linalg.solve(M, J.T @ (D * r_star))
        aref = J @ a_star - r_star
        cg = oracle.forward_cg(M, J, a0, aref, D, max_iter=20 * n, tol=1e-12)
        assert cg["status"] == oracle.ST_CONVERGED
        assert cg["active"].all()
        assert np.abs(cg["a"] - a_star).max() <= 1e-10 * np.abs(a_star).max(), n


def test_no_contacts_returns_a0():
    b = synth.uniform_batch(3, 7, 0, 9)
    for i in range(3):
        cg = oracle.forward_cg(b.M[i], b.J[i], b.a0[i], b.aref[i], b.D[i], max_iter=10)
        assert cg["status"] == oracle.ST_CONVERGED and cg["iters"] == 0
        assert np.array_equal(cg["a"], b.a0[i])


def test_cg_reaches_the_newton_minimiser():
    for (B, n, nc, seed) in ((24, 9, 16, 20260725), (24, 6, 4, 41), (12, 18, 32, 3)):
        b = synth.uniform_batch(B, n, nc, seed)
        for i in range(B):
            M, J = b.M[i].reshape(n, n), b.J[i].reshape(-1, n)
            nw = oracle.forward(M, J, b.a0[i], b.aref[i], b.D[i], max_iter=80, tol=1e-13)
            cg = oracle.forward_cg(M, J, b.a0[i], b.aref[i], b.D[i], max_iter=20000, tol=1e-11)
            assert nw["status"] == oracle.ST_CONVERGED and cg["status"] == oracle.ST_CONVERGED
            F = _stationarity(M, J, b.a0[i], b.aref[i], b.D[i], cg["a"])
            scale = np.trace(M) * (1 + np.abs(cg["a"]).max())
            assert np.linalg.norm(F) <= 1e-9 * scale, (n, i)
            assert np.array_equal(cg["active"], nw["active"]), (n, i)
            assert np.abs(cg["a"] - nw["a"]).max() <= 1e-8 * np.abs(nw["a"]).max(), (n, i)


def test_packed_equals_single():
    pb = synth.uneven_batch(20, (3, 9, 18), 24, seed=8)
    P = oracle.Packed(pb.nv, pb.nrows, pb.M, pb.J, pb.a0, pb.aref, pb.D)
    out = P.forward_cg(max_iter=3000, tol=1e-12)
    for i in range(20):
        d = pb.get(i)
        one = oracle.forward_cg(d["M"], d["J"], d["a0"], d["aref"], d["D"], max_iter=3000, tol=1e-12)
        assert out["status"][i] == one["status"] and out["iters"][i] == one["iters"]
        assert np.array_equal(out["a"][pb.off_n[i]:pb.off_n[i + 1]], one["a"])
        assert np.array_equal(out["active"][pb.off_m[i]:pb.off_m[i + 1]].astype(bool), one["active"])
