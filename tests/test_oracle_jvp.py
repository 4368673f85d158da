"""Pins of the oracle's IFT Jacobian-vector products (eq. 15, forward mode):
central finite differences of the oracle's own converged solution along
random directions of (a0, aref), duality with the separately pinned IFT VJP
(<abar, J da> = <a0bar, da0> + <arefbar, daref>), the closed form with no
contacts (da = da0), and the packed-batch entry against the single-instance
one."""
import numpy as np

import oracle
from paper_2607_24959_amd import synth


def _solve(b, i, a0=None, aref=None):
    r = oracle.forward(b.M[i], b.J[i], b.a0[i] if a0 is None else a0,
                       b.aref[i] if aref is None else aref, b.D[i], max_iter=80, tol=1e-13)
    assert r["status"] == oracle.ST_CONVERGED
    return r


def test_jvp_matches_central_fd():
    b = synth.uniform_batch(24, 6, 4, 777)
    rng = np.random.default_rng(1)
    eps = 1e-6
    checked = 0
    for i in range(b.B):
        base = _solve(b, i)
        d0 = rng.standard_normal((3, b.n))
        dr = rng.standard_normal((3, b.m))
        da = oracle.ift_jvp(b.M[i], b.J[i], b.D[i], base["active"], d0, dr)
        for k in range(3):
            p = _solve(b, i, b.a0[i] + eps * d0[k], b.aref[i] + eps * dr[k])
            q = _solve(b, i, b.a0[i] - eps * d0[k], b.aref[i] - eps * dr[k])
            if not (np.array_equal(p["active"], base["active"]) and
                    np.array_equal(q["active"], base["active"])):
                continue     # the active set changed within +-eps: no derivative there
            fd = (p["a"] - q["a"]) / (2 * eps)
            assert np.linalg.norm(fd - da[k]) <= 1e-6 * max(np.linalg.norm(da[k]), 1e-8), (i, k)
            checked += 1
    assert checked >= 60


def test_jvp_is_the_adjoint_of_the_vjp():
    b = synth.uniform_batch(16, 9, 8, 31)
    rng = np.random.default_rng(2)
    for i in range(b.B):
        base = _solve(b, i)
        d0 = rng.standard_normal((2, b.n))
        dr = rng.standard_normal((2, b.m))
        da = oracle.ift_jvp(b.M[i], b.J[i], b.D[i], base["active"], d0, dr)
        abar = rng.standard_normal(b.n)
        g = oracle.ift_vjp(b.M[i], b.J[i], b.a0[i], b.aref[i], b.D[i], base["a"], abar,
                           active=base["active"])
        for k in range(2):
            lhs = abar @ da[k]
            rhs = g["a0"] @ d0[k] + g["aref"] @ dr[k]
            assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + np.linalg.norm(abar) * np.linalg.norm(da[k])), i


def test_no_contacts_gives_the_tangent_of_a0():
    b = synth.uniform_batch(4, 5, 0, 3)
    rng = np.random.default_rng(3)
    for i in range(b.B):
        d0 = rng.standard_normal((4, b.n))
        da = oracle.ift_jvp(b.M[i], b.J[i], b.D[i], np.zeros(0, np.uint8), d0, None)
        assert np.allclose(da, d0, rtol=1e-12, atol=1e-12)


def test_packed_entry_matches_single_instance():
    pb = synth.uneven_batch(12, (3, 9, 18), 16, seed=5)
    P = oracle.Packed(pb.nv, pb.nrows, pb.M, pb.J, pb.a0, pb.aref, pb.D, pb.abar)
    fw = P.forward(max_iter=80, tol=1e-12)
    k = 3
    rng = np.random.default_rng(4)
    d0 = rng.standard_normal(k * int(pb.off_n[-1]))
    dr = rng.standard_normal(k * int(pb.off_m[-1]))
    da = P.ift_jvp(fw["active"], k, d0, dr)
    for i in range(pb.B):
        d = pb.get(i)
        n, m = d["n"], d["m"]
        act = fw["active"][pb.off_m[i]:pb.off_m[i + 1]]
        ref = oracle.ift_jvp(d["M"], d["J"], d["D"], act,
                             d0[k * pb.off_n[i]:k * pb.off_n[i] + k * n].reshape(k, n),
                             dr[k * pb.off_m[i]:k * pb.off_m[i] + k * m].reshape(k, m), k=k)
        got = da[k * pb.off_n[i]:k * pb.off_n[i] + k * n].reshape(k, n)
        assert np.array_equal(got, ref), i
