"""Pins of the oracle's unrolled-trace VJP.

Unrolled reverse mode differentiates the executed K-step solver trace, so
its reference is the central finite difference of the K-step map with the
whole trace (every active set, line-search piece and stop decision) held
fixed.  Once the trace contains a full step on the final piece the K-step
map no longer depends on earlier iterates and the unrolled gradient equals
the IFT one (Sec. III-B eqs. 11-14 and Sec. III-D); with a short trace it
does not.
"""
import numpy as np
import pytest

import oracle
from oracle import fd
from paper_2607_24959_amd import synth

KEYS = ("M", "J", "a0", "aref", "D")


@pytest.mark.parametrize("K", [1, 2, 3, 5])
def test_unrolled_matches_fd_of_k_step_map(K):
    rng = np.random.default_rng(19 + K)
    n_valid = 0
    for i in range(6):
        d = synth.instance(51, i, 6, 4)
        abar = d["abar"]
        g = oracle.unrolled_vjp(*(d[k] for k in KEYS), abar, K=K, tol=1e-13)
        fw = oracle.forward(*(d[k] for k in KEYS), max_iter=K, tol=1e-13)
        assert np.array_equal(g["a"], fw["a"])
        for key in KEYS:
            E = fd.random_direction(rng, d[key], symmetric=(key == "M"))
            ana = float(np.sum(g[key] * E))
            # epsilon sweep: the K-step map carries rounding noise from its large first
            # steps and curvature from alpha = -b/c, so the plateau of the sweep is the
            # reference (valid samples only: the whole trace must stay fixed)
            errs = []
            for eps in (3e-3, 1e-3, 3e-4, 1e-4, 3e-5, 1e-5, 1e-6):
                num, valid = fd.fd_directional(d, key, E, abar, eps=eps, max_iter=K, tol=1e-13,
                                               unrolled=True)
                if valid:
                    errs.append(abs(num - ana))
            if not errs:
                continue
            assert min(errs) <= 1e-6 * (abs(ana) + 1e-3 * np.linalg.norm(g[key]) + 1e-8), (key, K)
            n_valid += 1
    assert n_valid >= 15


def test_converged_trace_equals_ift():
    for i in range(8):
        d = synth.instance(52, i, 9, 16)
        fw = oracle.forward(*(d[k] for k in KEYS), max_iter=100, tol=1e-13)
        assert fw["status"] == oracle.ST_CONVERGED
        ift = oracle.ift_vjp(*(d[k] for k in KEYS), fw["a"], d["abar"], active=fw["active"])
        un = oracle.unrolled_vjp(*(d[k] for k in KEYS), d["abar"], K=100, tol=1e-13)
        assert un["status"] == oracle.ST_CONVERGED
        for k in KEYS:
            assert np.allclose(un[k], ift[k], rtol=1e-7, atol=1e-9 * np.abs(ift[k]).max()), k


def test_short_trace_differs_from_ift():
    diffs = []
    for i in range(8):
        d = synth.instance(53, i, 6, 4)
        fw = oracle.forward(*(d[k] for k in KEYS), max_iter=100, tol=1e-13)
        ift = oracle.ift_vjp(*(d[k] for k in KEYS), fw["a"], d["abar"], active=fw["active"])
        un = oracle.unrolled_vjp(*(d[k] for k in KEYS), d["abar"], K=1, tol=1e-13)
        diffs.append(np.linalg.norm(un["aref"] - ift["aref"]) / np.linalg.norm(ift["aref"]))
    assert np.median(diffs) > 1e-2


def test_k_zero_is_identity():
    d = synth.instance(54, 0, 5, 3)
    g = oracle.unrolled_vjp(*(d[k] for k in KEYS), d["abar"], K=0, tol=1e-13)
    assert np.array_equal(g["a"], d["a0"])
    assert np.array_equal(g["a0"], d["abar"])
    for k in ("aref", "J", "D", "M"):
        assert not np.any(g[k])
