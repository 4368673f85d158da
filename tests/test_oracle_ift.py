"""Pins of the oracle's IFT VJP (Sec. III-C, eq. 17).

Checked against: central finite differences of the converged solution map
with the contact schedule held fixed (the paper's validation protocol), a
hand-worked golden case, exact identities that follow from invariances of
the minimiser, and closed forms (no contacts; every row active, where a
library autograd of a dense linear solve is the reference).
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import fd
from paper_2607_24959_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
KEYS = ("M", "J", "a0", "aref", "D")


def _grads(d, abar, **kw):
    res = oracle.forward(*(d[k] for k in KEYS), max_iter=100, tol=1e-13)
    assert res["status"] == oracle.ST_CONVERGED
    g = oracle.ift_vjp(*(d[k] for k in KEYS), res["a"], abar, active=res["active"])
    return res, g


def test_golden_cases():
    for name in ("scalar_contact.json", "two_row_inactive.json"):
        g = json.load(open(os.path.join(GOLD, name)))
        d = {k: np.array(g[k], dtype=float) for k in KEYS}
        _, gr = _grads(d, np.array(g["abar"]))
        for k in KEYS:
            assert np.allclose(gr[k], np.array(g["grad"][k]), rtol=1e-13, atol=1e-14), k


@pytest.mark.parametrize("n,nc", [(6, 4), (9, 16)])
def test_central_fd_every_input(n, nc):
    rng = np.random.default_rng(7)
    n_valid = 0
    for i in range(8):
        d = synth.instance(41, i, n, nc)
        abar = d["abar"]
        _, g = _grads(d, abar)
        for key in KEYS:
            E = fd.random_direction(rng, d[key], symmetric=(key == "M"))
            num, valid = fd.fd_directional(d, key, E, abar, eps=1e-6, max_iter=100, tol=1e-13)
            if not valid:
                continue
            ana = float(np.sum(g[key] * E))
            assert abs(num - ana) <= 1e-5 * (abs(ana) + 1e-3 * np.linalg.norm(g[key]) + 1e-8), key
            n_valid += 1
    assert n_valid >= 30


def test_fd_epsilon_plateau():
    d = synth.instance(42, 0, 6, 4)
    abar = d["abar"]
    _, g = _grads(d, abar)
    E = np.random.default_rng(1).standard_normal(d["aref"].shape)
    ana = float(np.sum(g["aref"] * E))
    for eps in (1e-4, 1e-5, 1e-6, 1e-7, 1e-8):
        num, valid = fd.fd_directional(d, "aref", E, abar, eps=eps, max_iter=100, tol=1e-13)
        assert valid
        assert abs(num - ana) <= 1e-4 * abs(ana) + 1e-7


def test_invariance_identities():
    for i in range(10):
        d = synth.instance(43, i, 9, 16)
        res, g = _grads(d, d["abar"])
        # (i) translation a0 + delta, aref + J delta -> a* + delta
        assert np.allclose(g["a0"] + d["J"].T @ g["aref"], d["abar"], rtol=1e-9, atol=1e-9)
        # (ii) scaling (M, D) -> c (M, D) leaves a* unchanged
        s = np.sum(g["M"] * d["M"]) + np.sum(g["D"] * d["D"])
        scale = np.abs(g["M"] * d["M"]).sum() + np.abs(g["D"] * d["D"]).sum()
        assert abs(s) <= 1e-9 * scale
        # (iii) row scaling (J_i, aref_i, D_i) -> (c J_i, c aref_i, D_i / c^2)
        row = np.sum(g["J"] * d["J"], axis=1) + g["aref"] * d["aref"] - 2 * g["D"] * d["D"]
        rscale = np.abs(g["J"] * d["J"]).sum(1) + np.abs(g["aref"] * d["aref"]) + 2 * np.abs(g["D"] * d["D"])
        assert np.all(np.abs(row) <= 1e-9 * (rscale + 1e-12))


def test_no_contacts_closed_form():
    d = synth.instance(44, 0, 7, 0)
    _, g = _grads(d, d["abar"])
    assert np.allclose(g["a0"], d["abar"], rtol=1e-13, atol=1e-13)
    lam = np.linalg.solve(d["M"], d["abar"])
    assert np.allclose(g["M"], np.zeros((7, 7)), atol=1e-12)  # a* = a0 so M does not enter
    assert np.allclose(lam, g["lam"], rtol=1e-12)


def test_all_active_matches_library_autograd():
    d = synth.instance(45, 0, 6, 4)
    G = d["J"] @ np.linalg.solve(d["M"], d["J"].T)
    m = d["J"].shape[0]
    d["aref"] = d["J"] @ d["a0"] + (np.eye(m) + G * d["D"][None, :]) @ np.full(m, 10.0)
    res, g = _grads(d, d["abar"])
    assert res["active"].all()
    t = {k: torch.tensor(d[k], dtype=torch.float64, requires_grad=True) for k in KEYS}
    H = t["M"] + t["J"].T @ (t["D"][:, None] * t["J"])
    rhs = t["M"] @ t["a0"] + t["J"].T @ (t["D"] * t["aref"])
    a = torch.linalg.solve(H, rhs)
    (a @ torch.tensor(d["abar"], dtype=torch.float64)).backward()
    for k in KEYS:
        assert np.allclose(g[k], t[k].grad.numpy(), rtol=1e-9, atol=1e-10), k
