"""Pins of the oracle's round-cone (elliptic) contact solve (Sec. III-A, eqs. 2,
3 and 5: s is the R^{-1}-weighted squared distance to the dual cone K*):

* s at random points against a brute-force projection onto K* (a search over
  the cone's boundary rays), its gradient and Hessian against central
  differences of s and of the gradient;
* the regularised force -ds/du lies in the friction cone K, the projection
  z* = u - R ds/du lies in K*, and the two are complementary (eq. 3's duality);
* mu = 0 turns the cone into the half-space of the normal rows alone: the
  solve and its VJP equal the separately pinned pyramid oracle on those rows;
* the forward's result minimises L: F(a*) = 0, and L built on the brute-force
  projection does not decrease in any of 64 random directions;
* the IFT VJP of every input (M, J, a0, aref, D_N, D_T, mu) against central
  finite differences of the oracle's converged solution.
"""
import numpy as np
import pytest
from scipy import optimize

import oracle
from paper_2607_24959_amd import synth


def _brute_s(u, dn, dt, mu):
    """min over z in K* = {z_N >= mu |z_T|} of 1/2 (u - z)^T diag(dn, dt, dt) (u - z),
    by direct search: the minimiser is u itself (u in K*), or lies on K*'s boundary
    z = (mu rho, rho cos phi, rho sin phi), rho >= 0 (rho = 0 is the apex).  For a fixed
    angle the best rho solves a scalar quadratic; the angle is searched on a grid and
    refined by a bounded scalar minimisation."""
    W = np.array([dn, dt, dt])
    if u[0] >= mu * np.hypot(u[1], u[2]):
        return 0.0

    def on_ray(phi):
        c, s_ = np.cos(phi), np.sin(phi)
        rho = max(0.0, (dn * mu * u[0] + dt * (u[1] * c + u[2] * s_)) / (dn * mu * mu + dt))
        z = np.array([mu * rho, rho * c, rho * s_])
        return 0.5 * np.sum(W * (u - z) ** 2)

    grid = np.linspace(0.0, 2 * np.pi, 721)
    vals = np.array([on_ray(p) for p in grid])
    k = int(np.argmin(vals))
    r = optimize.minimize_scalar(on_ray, bounds=(grid[max(k - 1, 0)], grid[min(k + 1, 720)]),
                                 method="bounded", options=dict(xatol=1e-14))
    return min(vals.min(), r.fun)


def _rand_points(rng, k):
    for _ in range(k):
        u = rng.standard_normal(3) * rng.choice([0.1, 1.0, 10.0])
        dn = 10 ** rng.uniform(-1, 2)
        dt = dn * 10 ** rng.uniform(-1, 1)
        mu = rng.uniform(0.1, 1.5)
        yield u, dn, dt, mu


def test_block_value_against_brute_projection():
    rng = np.random.default_rng(3)
    zones = set()
    for u, dn, dt, mu in _rand_points(rng, 60):
        z, w, G, s = oracle.ell_block(u, dn, dt, mu)
        zones.add(z)
        sb = _brute_s(u, dn, dt, mu)
        assert abs(s - sb) <= 1e-8 * (1 + abs(sb)), (u, dn, dt, mu, s, sb)
    assert zones == {0, 1, 2}


def test_block_gradient_and_hessian_by_differences():
    rng = np.random.default_rng(4)
    for u, dn, dt, mu in _rand_points(rng, 80):
        z, w, G, s = oracle.ell_block(u, dn, dt, mu)
        h = 1e-6 * (1 + np.abs(u).max())
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            zp, wp, _, sp = oracle.ell_block(u + e, dn, dt, mu)
            zm, wm, _, sm = oracle.ell_block(u - e, dn, dt, mu)
            if zp != z or zm != z:
                continue        # a zone boundary within h: s is C^1 only there
            assert abs((sp - sm) / (2 * h) - w[k]) <= 1e-6 * (1 + np.abs(w).max())
            assert np.abs((wp - wm) / (2 * h) - G[:, k]).max() <= 1e-5 * (1 + np.abs(G).max())
        assert np.allclose(G, G.T)
        assert np.linalg.eigvalsh(G).min() >= -1e-12 * (1 + np.abs(G).max())


def test_force_in_cone_and_complementary():
    rng = np.random.default_rng(5)
    for u, dn, dt, mu in _rand_points(rng, 200):
        z, w, G, s = oracle.ell_block(u, dn, dt, mu)
        lam = -w                                   # regularised contact force
        zs = u - w / np.array([dn, dt, dt])        # the projection onto K*
        scale = 1 + np.abs(u).max() * max(dn, dt)
        assert lam[0] >= -1e-12 * scale
        assert np.hypot(lam[1], lam[2]) <= mu * lam[0] + 1e-10 * scale
        assert zs[0] >= mu * np.hypot(zs[1], zs[2]) - 1e-10 * (1 + np.abs(u).max())
        assert abs(lam @ zs) <= 1e-9 * scale * (1 + np.abs(u).max())


def test_mu_zero_is_the_pyramid_on_the_normal_rows():
    b = synth.elliptic_batch(12, 6, 5, 11)
    for i in range(12):
        mu0 = np.zeros(b.nc)
        r = oracle.forward_ell(b.M[i], b.J[i], b.a0[i], b.aref[i], b.dn[i], b.dt[i], mu0,
                               max_iter=80, tol=1e-13)
        Jn, arn = b.J[i][0::3], b.aref[i][0::3]
        p = oracle.forward(b.M[i], Jn, b.a0[i], arn, b.dn[i], max_iter=80, tol=1e-13)
        assert r["status"] == p["status"] == oracle.ST_CONVERGED
        assert np.abs(r["a"] - p["a"]).max() <= 1e-12 * np.abs(p["a"]).max()
        assert np.array_equal(r["zone"] != 0, p["active"])
        g = oracle.ift_vjp_ell(b.M[i], b.J[i], b.a0[i], b.aref[i], b.dn[i], b.dt[i], mu0, r["a"],
                               b.abar[i])
        q = oracle.ift_vjp(b.M[i], Jn, b.a0[i], arn, b.dn[i], p["a"], b.abar[i], active=p["active"])
        tol = lambda x: 1e-10 * (1 + np.abs(x).max())
        assert np.abs(g["a0"] - q["a0"]).max() <= tol(q["a0"])
        assert np.abs(g["aref"][0::3] - q["aref"]).max() <= tol(q["aref"])
        assert np.abs(g["J"][0::3] - q["J"]).max() <= tol(q["J"])
        assert np.abs(g["dn"] - q["D"]).max() <= tol(q["D"])
        assert np.abs(g["M"] - q["M"]).max() <= tol(q["M"])
        # the tangential rows carry no force when mu = 0
        assert np.abs(g["aref"][1::3]).max() <= tol(q["aref"])
        assert np.abs(g["dt"]).max() <= tol(q["D"])


def test_forward_minimises_L():
    """F(a*) = 0, and L built on the brute-force projection does not decrease
    along 64 random directions from a* (L is convex, so a* is its minimiser)."""
    b = synth.elliptic_batch(6, 3, 2, 21)
    rng = np.random.default_rng(21)
    for i in range(6):
        args = (b.M[i], b.J[i], b.a0[i], b.aref[i], b.dn[i], b.dt[i], b.mu[i])
        r = oracle.forward_ell(*args, max_iter=80, tol=1e-13)
        assert r["status"] == oracle.ST_CONVERGED
        Lv, F = oracle.ell_objective(*args, r["a"])
        assert np.linalg.norm(F) <= 1e-8 * np.trace(b.M[i]) * (1 + np.abs(r["a"]).max())

        def L_brute(a):
            d = a - b.a0[i]
            u = b.J[i] @ a - b.aref[i]
            return 0.5 * d @ b.M[i] @ d + sum(
                _brute_s(u[3 * c:3 * c + 3], b.dn[i][c], b.dt[i][c], b.mu[i][c])
                for c in range(b.nc))

        L0 = L_brute(r["a"])
        assert abs(L0 - Lv) <= 1e-9 * (1 + abs(Lv))
        eps = 1e-3 * (1 + np.abs(r["a"]).max())
        for _ in range(64):
            d = rng.standard_normal(b.n)
            d *= eps / np.linalg.norm(d)
            assert L_brute(r["a"] + d) >= L0 - 1e-10 * (1 + abs(L0))
            assert L_brute(r["a"] - d) >= L0 - 1e-10 * (1 + abs(L0))


@pytest.mark.parametrize("seed", [7, 8])
def test_vjp_every_input_against_central_fd(seed):
    b = synth.elliptic_batch(6, 6, 4, seed)
    rng = np.random.default_rng(seed)
    names = ("M", "J", "a0", "aref", "dn", "dt", "mu")
    checked = 0
    for i in range(6):
        args = [b.M[i], b.J[i], b.a0[i], b.aref[i], b.dn[i], b.dt[i], b.mu[i]]
        r = oracle.forward_ell(*args, max_iter=80, tol=1e-14)
        g = oracle.ift_vjp_ell(*args, r["a"], b.abar[i])
        for k, name in enumerate(names):
            X = np.array(args[k], dtype=float)
            dX = rng.standard_normal(X.shape)
            if name == "M":
                dX = dX + dX.T
            eps = 1e-6 * max(1.0, np.abs(X).max())

            def sol(sg):
                A = list(args)
                A[k] = X + sg * eps * dX
                return oracle.forward_ell(*A, max_iter=80, tol=1e-14)

            ap, am = sol(1), sol(-1)
            if not (np.array_equal(ap["zone"], r["zone"]) and np.array_equal(am["zone"], r["zone"])):
                continue
            fd = b.abar[i] @ (ap["a"] - am["a"]) / (2 * eps)
            an = float(np.sum(np.asarray(g[name]).reshape(X.shape) * dX))
            assert abs(fd - an) <= 1e-5 * (abs(an) + 1e-3 * np.abs(g[name]).max() * np.abs(dX).sum()), \
                (i, name, fd, an)
            checked += 1
    assert checked >= 30
