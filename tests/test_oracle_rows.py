"""Pins of the oracle's mixed-row solve (one-sided, equality and friction-loss
rows; Sec. III-A's other regularised constraint rows):

* one-sided rows alone are the pyramid oracle (solve and VJP);
* brute force on tiny instances: every assignment of zones (one-sided: off /
  quadratic; equality: quadratic; friction loss: quadratic / saturated at +f /
  at -f) gives one linear system; exactly one solution is consistent with its
  own zones, and it is the oracle's a*;
* limits of the friction bound: f -> infinity turns a friction-loss row into
  an equality row, f = 0 removes it;
* the IFT VJP of every input (M, J, a0, aref, D, f) against central FD.
"""
import itertools

import numpy as np

import oracle
from paper_2607_24959_amd import synth


def _zone(kind, r, D, f):
    if kind == 0:
        return 1 if r < 0 else 0
    if kind == 1:
        return 1
    return 2 if r > f / D else (3 if r < -f / D else 1)


def test_one_sided_rows_are_the_pyramid():
    b = synth.mixed_batch(10, 6, 4, 0, 0, 3)
    for i in range(10):
        r = oracle.forward_rows(b.M[i], b.J[i], b.a0[i], b.aref[i], b.D[i], b.kind[i], b.floss[i],
                                max_iter=60, tol=1e-13)
        p = oracle.forward(b.M[i], b.J[i], b.a0[i], b.aref[i], b.D[i], max_iter=60, tol=1e-13)
        assert r["status"] == p["status"] == oracle.ST_CONVERGED and r["iters"] == p["iters"]
        assert np.abs(r["a"] - p["a"]).max() <= 1e-12 * np.abs(p["a"]).max()
        assert np.array_equal(r["zone"] == 1, p["active"])
        g = oracle.ift_vjp_rows(b.M[i], b.J[i], b.a0[i], b.aref[i], b.D[i], b.kind[i], b.floss[i],
                                r["a"], b.abar[i])
        q = oracle.ift_vjp(b.M[i], b.J[i], b.a0[i], b.aref[i], b.D[i], p["a"], b.abar[i],
                           active=p["active"])
        for k in ("a0", "aref", "J", "D", "M"):
            assert np.abs(g[k] - q[k]).max() <= 1e-10 * (1 + np.abs(q[k]).max()), k
        assert np.all(g["floss"] == 0)


def test_brute_force_zone_enumeration():
    b = synth.mixed_batch(12, 3, 1, 1, 2, 11)
    for i in range(12):
        M, J, a0, aref, D, kind, f = (b.M[i], b.J[i], b.a0[i], b.aref[i], b.D[i], b.kind[i],
                                      b.floss[i])
        choices = [(0, 1) if k == 0 else ((1,) if k == 1 else (1, 2, 3)) for k in kind]
        found = []
        for zs in itertools.product(*choices):
            zs = np.array(zs)
            g = np.where(zs == 1, D, 0.0)
            rhs = M @ a0 + J.T @ (g * aref) - J.T @ (np.where(zs == 2, f, 0.0) -
                                                      np.where(zs == 3, f, 0.0))
            a = np.linalg.solve(M + J.T @ (g[:, None] * J), rhs)
            r = J @ a - aref
            if all(_zone(kind[k], r[k], D[k], f[k]) == zs[k] for k in range(len(kind))):
                found.append((zs, a))
        assert len(found) == 1, (i, len(found))
        o = oracle.forward_rows(M, J, a0, aref, D, kind, f, max_iter=60, tol=1e-13)
        assert o["status"] == oracle.ST_CONVERGED
        assert np.array_equal(o["zone"], found[0][0]), i
        assert np.abs(o["a"] - found[0][1]).max() <= 1e-10 * np.abs(found[0][1]).max(), i


def test_friction_bound_limits():
    b = synth.mixed_batch(8, 6, 3, 0, 3, 13)
    for i in range(8):
        M, J, a0, aref, D, kind = b.M[i], b.J[i], b.a0[i], b.aref[i], b.D[i], b.kind[i]
        big = np.where(kind == 2, 1e12, 0.0)
        r_big = oracle.forward_rows(M, J, a0, aref, D, kind, big, max_iter=60, tol=1e-13)
        eq = np.where(kind == 2, 1, kind).astype(np.uint8)
        r_eq = oracle.forward_rows(M, J, a0, aref, D, eq, np.zeros_like(big), max_iter=60, tol=1e-13)
        assert np.abs(r_big["a"] - r_eq["a"]).max() <= 1e-9 * np.abs(r_eq["a"]).max()
        r_zero = oracle.forward_rows(M, J, a0, aref, D, kind, np.zeros_like(big), max_iter=60,
                                     tol=1e-13)
        keep = kind != 2
        r_rm = oracle.forward(M, J[keep], a0, aref[keep], D[keep], max_iter=60, tol=1e-13)
        assert np.abs(r_zero["a"] - r_rm["a"]).max() <= 1e-10 * np.abs(r_rm["a"]).max()


def test_vjp_every_input_against_central_fd():
    b = synth.mixed_batch(6, 6, 3, 2, 3, 17)
    rng = np.random.default_rng(17)
    names = ("M", "J", "a0", "aref", "D", "floss")
    checked = 0
    for i in range(6):
        args = dict(M=b.M[i], J=b.J[i], a0=b.a0[i], aref=b.aref[i], D=b.D[i], floss=b.floss[i])
        call = lambda A: oracle.forward_rows(A["M"], A["J"], A["a0"], A["aref"], A["D"], b.kind[i],
                                             A["floss"], max_iter=60, tol=1e-14)
        r = call(args)
        g = oracle.ift_vjp_rows(args["M"], args["J"], args["a0"], args["aref"], args["D"], b.kind[i],
                                args["floss"], r["a"], b.abar[i])
        for name in names:
            X = np.array(args[name], dtype=float)
            dX = rng.standard_normal(X.shape)
            if name == "M":
                dX = dX + dX.T
            if name == "floss":
                dX = dX * (b.kind[i] == 2)
            eps = 1e-6 * max(1.0, np.abs(X).max())
            sols = []
            for sg in (1, -1):
                A = dict(args)
                A[name] = X + sg * eps * dX
                sols.append(call(A))
            if not all(np.array_equal(s["zone"], r["zone"]) for s in sols):
                continue
            fd = b.abar[i] @ (sols[0]["a"] - sols[1]["a"]) / (2 * eps)
            an = float(np.sum(g[name].reshape(X.shape) * dX))
            assert abs(fd - an) <= 1e-5 * (abs(an) + 1e-6 * np.abs(g[name]).max() * np.abs(dX).sum()), \
                (i, name, fd, an)
            checked += 1
    assert checked >= 25
