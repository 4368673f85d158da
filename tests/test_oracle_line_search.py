"""Pins of the oracle's exact line search (Sec. III-B, eq. 10).

The step must be the exact minimiser of phi(t) = L(a + t p), where L is the
reduced objective of eq. 5.  The reference here never looks at breakpoints:
it evaluates L itself on a dense grid and refines with golden-section
search, then checks the oracle's sort-and-scan result and its piece.
"""
import json
import os

import numpy as np

import oracle
from paper_2607_24959_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
KEYS = ("M", "J", "a0", "aref", "D")


def _L(d, a):
    r = d["J"] @ a - d["aref"]
    e = a - d["a0"]
    return 0.5 * e @ d["M"] @ e + 0.5 * np.sum(d["D"] * np.minimum(r, 0.0) ** 2)


def _golden_min(f, lo, hi, iters=200):
    g = (np.sqrt(5) - 1) / 2
    x1, x2 = hi - g * (hi - lo), lo + g * (hi - lo)
    f1, f2 = f(x1), f(x2)
    for _ in range(iters):
        if f1 < f2:
            hi, x2, f2 = x2, x1, f1
            x1 = hi - g * (hi - lo)
            f1 = f(x1)
        else:
            lo, x1, f1 = x1, x2, f2
            x2 = lo + g * (hi - lo)
            f2 = f(x2)
    return 0.5 * (lo + hi)


def test_golden_two_rows():
    g = json.load(open(os.path.join(GOLD, "line_search_two_rows.json")))
    d = {k: np.array(g[k], dtype=float) for k in KEYS}
    alpha, Ap, _ = oracle.line_search(*(d[k] for k in KEYS), np.array(g["a"]), np.array(g["p"]))
    assert abs(alpha - g["alpha"]) < 1e-15
    assert Ap.tolist() == g["piece"]


def test_exact_minimiser_along_newton_and_random_directions():
    rng = np.random.default_rng(17)
    checked = 0
    for i in range(40):
        d = synth.instance(31, i, 9, 16)
        # a point along the way, and both a Newton direction and a random descent direction
        a = d["a0"] + rng.normal(0, 20, 9)
        r = d["J"] @ a - d["aref"]
        A = r < 0
        F = d["M"] @ (a - d["a0"]) + d["J"].T @ (d["D"] * A * r)
        H = d["M"] + d["J"].T @ ((d["D"] * A)[:, None] * d["J"])
        for p in (-np.linalg.solve(H, F), -F / np.linalg.norm(F) * rng.uniform(1, 30)):
            alpha, Ap, q = oracle.line_search(*(d[k] for k in KEYS), a, p)
            f = lambda t: _L(d, a + t * p)
            ts = np.linspace(0, 4 * max(alpha, 1.0), 4001)
            vals = np.array([f(t) for t in ts])
            k = int(np.argmin(vals))
            lo, hi = ts[max(k - 1, 0)], ts[min(k + 1, len(ts) - 1)]
            t_ref = _golden_min(f, lo, hi)
            assert alpha > 0
            assert abs(alpha - t_ref) <= 1e-6 * (1 + t_ref)
            assert f(alpha) <= f(t_ref) + 1e-12 * (1 + abs(f(t_ref)))
            # the reported piece is the active set strictly inside it
            z = r + alpha * q
            clear = np.abs(z) > 1e-12 * (1 + np.abs(r))
            assert np.array_equal(Ap[clear], (z < 0)[clear])
            checked += 1
    assert checked == 80


def test_no_rows_gives_unit_newton_step():
    d = synth.instance(3, 0, 4, 0)
    a = d["a0"] + 1.0
    p = -(a - d["a0"])
    alpha, _, _ = oracle.line_search(*(d[k] for k in KEYS), a, p)
    assert abs(alpha - 1.0) < 1e-14
