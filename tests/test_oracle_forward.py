"""Pins of the oracle's forward solve against what the mathematics fixes.

a* is the unique minimiser of the strictly convex piecewise quadratic of
Sec. III-A (eq. 5, pyramidal rows), i.e. the unique root of the stationarity
residual (eqs. 6-7).  These tests check the oracle's Newton + exact line
search result against: brute-force active-set enumeration, hand-worked and
closed-form cases, the root condition and H > 0 (eq. 9), independence of the
starting point (eq. 14), and invariances of the minimiser.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2607_24959_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
KEYS = ("M", "J", "a0", "aref", "D")


def _inst(seed, i, n, nc):
    return synth.instance(seed, i, n, nc)


def _solve(d, **kw):
    kw.setdefault("max_iter", 100)
    kw.setdefault("tol", 1e-12)
    return oracle.forward(*(d[k] for k in KEYS), **kw)


def _F(d, a):
    r = d["J"] @ a - d["aref"]
    return d["M"] @ (a - d["a0"]) + d["J"].T @ (d["D"] * np.minimum(r, 0.0))


def _rel(x, y):
    return np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-30)


@pytest.mark.parametrize("n,nc", [(6, 4), (3, 2), (1, 3), (2, 4)])
def test_brute_force_enumeration(n, nc):
    for i in range(6):
        d = _inst(101, i, n, nc)
        res = _solve(d)
        assert res["status"] == oracle.ST_CONVERGED
        a_bf, S_bf, n_cons, _ = brute.enumerate_solutions(*(d[k] for k in KEYS))
        assert n_cons == 1, "uniqueness: exactly one consistent active set"
        assert _rel(res["a"], a_bf) < 1e-10
        assert np.array_equal(res["active"], S_bf)


def test_golden_scalar_contact():
    g = json.load(open(os.path.join(GOLD, "scalar_contact.json")))
    d = {k: np.array(g[k], dtype=float) for k in KEYS}
    res = _solve(d)
    assert np.allclose(res["a"], g["a_star"], rtol=1e-14, atol=1e-14)
    assert res["active"].tolist() == g["active"]


def test_golden_two_rows_one_inactive():
    g = json.load(open(os.path.join(GOLD, "two_row_inactive.json")))
    d = {k: np.array(g[k], dtype=float) for k in KEYS}
    res = _solve(d)
    assert np.allclose(res["a"], g["a_star"], rtol=1e-14, atol=1e-14)
    assert res["active"].tolist() == g["active"]


def test_no_contacts_returns_a0():
    d = _inst(7, 0, 5, 0)
    res = _solve(d)
    assert res["status"] == oracle.ST_CONVERGED and res["iters"] == 0
    assert np.array_equal(res["a"], d["a0"])


def test_all_rows_active_is_one_linear_system():
    d = _inst(8, 0, 6, 4)
    # With every row active, r(a_S) = -(I + J M^-1 J^T D)^-1 (aref - J a0); choosing
    # aref - J a0 = (I + J M^-1 J^T D) 1 s puts every row at r = -s < 0, so the
    # all-active system's solution is consistent and therefore equals a*.
    G = d["J"] @ np.linalg.solve(d["M"], d["J"].T)
    m = d["J"].shape[0]
    d["aref"] = d["J"] @ d["a0"] + (np.eye(m) + G * d["D"][None, :]) @ np.full(m, 10.0)
    res = _solve(d)
    H = d["M"] + d["J"].T @ (d["D"][:, None] * d["J"])
    a_ls = np.linalg.solve(H, d["M"] @ d["a0"] + d["J"].T @ (d["D"] * d["aref"]))
    assert res["active"].all()
    assert _rel(res["a"], a_ls) < 1e-12


def test_scalar_formula_one_row():
    rng = np.random.default_rng(3)
    for _ in range(20):
        Mv, j, dd, rho, a0 = rng.uniform(0.5, 2), rng.normal(), rng.uniform(1, 100), rng.normal() * 3, rng.normal()
        d = dict(M=np.array([[Mv]]), J=np.array([[j]]), a0=np.array([a0]), aref=np.array([rho]),
                 D=np.array([dd]))
        if j * a0 - rho >= 0:
            expect = a0
        else:
            expect = (Mv * a0 + dd * j * rho) / (Mv + dd * j * j)
        res = _solve(d)
        assert abs(res["a"][0] - expect) <= 1e-13 * (1 + abs(expect))


def test_root_and_spd_newton_matrix():
    b = synth.uniform_batch(64, 9, 16, 55)
    for i in range(b.B):
        d = {k: getattr(b, k)[i] for k in KEYS}
        res = _solve(d, tol=1e-12)
        assert res["status"] == oracle.ST_CONVERGED
        a = res["a"]
        assert np.linalg.norm(_F(d, a)) <= 1e-9 * np.trace(d["M"])
        A = (d["J"] @ a - d["aref"]) < 0
        assert np.array_equal(A, res["active"])
        H = d["M"] + d["J"].T @ ((d["D"] * A)[:, None] * d["J"])
        assert np.linalg.eigvalsh(H).min() > 0


def test_independent_of_starting_point():
    rng = np.random.default_rng(11)
    for i in range(10):
        d = _inst(12, i, 9, 16)
        ref = _solve(d)
        other = _solve(d, a_init=rng.normal(0, 50, 9))
        assert ref["status"] == other["status"] == oracle.ST_CONVERGED
        assert _rel(other["a"], ref["a"]) < 1e-10
        assert np.array_equal(other["active"], ref["active"])


def test_invariances_of_the_minimiser():
    rng = np.random.default_rng(5)
    for i in range(6):
        d = _inst(13, i, 6, 4)
        a = _solve(d)["a"]
        m, n = d["J"].shape
        # (M, D) -> c (M, D)
        e = dict(d, M=3.7 * d["M"], D=3.7 * d["D"])
        assert _rel(_solve(e)["a"], a) < 1e-10
        # row permutation
        P = rng.permutation(m)
        e = dict(d, J=d["J"][P], aref=d["aref"][P], D=d["D"][P])
        assert _rel(_solve(e)["a"], a) < 1e-10
        # split every row into two copies with half the weight
        e = dict(d, J=np.vstack([d["J"], d["J"]]), aref=np.concatenate([d["aref"], d["aref"]]),
                 D=np.concatenate([d["D"], d["D"]]) / 2)
        assert _rel(_solve(e)["a"], a) < 1e-10
        # translation a0 + delta, aref + J delta -> a* + delta
        delta = rng.normal(0, 5, n)
        e = dict(d, a0=d["a0"] + delta, aref=d["aref"] + d["J"] @ delta)
        assert _rel(_solve(e)["a"], a + delta) < 1e-10
        # row scaling (J_i, aref_i, D_i) -> (c J_i, c aref_i, D_i / c^2)
        c = rng.uniform(0.3, 3.0, m)
        e = dict(d, J=d["J"] * c[:, None], aref=d["aref"] * c, D=d["D"] / c ** 2)
        assert _rel(_solve(e)["a"], a) < 1e-10


def test_iteration_cap_and_status_codes():
    d = _inst(14, 0, 9, 16)
    r0 = _solve(d, max_iter=0)
    assert r0["iters"] == 0 and r0["status"] == oracle.ST_MAXITER
    assert np.array_equal(r0["a"], d["a0"])
    r1 = _solve(d, max_iter=1)
    assert r1["iters"] == 1
    bad = dict(d)
    bad["aref"] = d["aref"].copy()
    bad["aref"][3] = np.nan
    assert _solve(bad)["status"] == oracle.ST_NONFINITE
    neg = dict(d, M=-np.eye(9))
    r = _solve(neg)
    assert r["status"] == oracle.ST_NOTSPD and np.isnan(r["a"]).all()


def test_batch_entry_matches_single_instances():
    pb = synth.uneven_batch(24, (3, 9, 18), 12, seed=21)
    P = oracle.Packed(pb.nv, pb.nrows, pb.M, pb.J, pb.a0, pb.aref, pb.D, pb.abar)
    out = P.forward(max_iter=50, tol=1e-12, threads=2)
    for i in range(pb.B):
        d = pb.get(i)
        res = _solve(d, max_iter=50, tol=1e-12)
        sl = slice(pb.off_n[i], pb.off_n[i + 1])
        assert np.array_equal(out["a"][sl], res["a"])
        assert out["iters"][i] == res["iters"] and out["status"][i] == res["status"]
