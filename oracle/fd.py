"""Central finite differences of the oracle's solution maps (test infrastructure).

Following the paper's validation protocol (Sec. III-D): every perturbation
must preserve the nominal contact schedule, so a sample is *valid* only when
the active set of the solution (for the converged map) or the whole executed
trace -- every A_k, every line-search piece A'_k, the number of steps and the
stop decision -- is identical at theta + eps E and theta - eps E.
"""
from __future__ import annotations

import numpy as np

from . import forward, ST_CONVERGED

KEYS = ("M", "J", "a0", "aref", "D")


def _perturbed(inst, key, E, s):
    out = {k: np.array(inst[k], dtype=np.float64, copy=True) for k in KEYS}
    out[key] = out[key] + s * E
    return out


def _signature(res, trace):
    sig = (res["status"], tuple(res["active"].tolist()))
    if trace:
        sig = sig + (res["iters"], res["A"].tobytes(), res["Ap"].tobytes())
    return sig


def fd_directional(inst, key, E, abar, eps=1e-6, max_iter=50, tol=1e-10, unrolled=False):
    """Return (d/deps [abar . a(theta + eps E)], valid).

    ``unrolled=False``: the converged solution map (needs status CONVERGED);
    ``unrolled=True``: the K-step map with K = ``max_iter`` and the full trace
    held fixed.
    """
    kw = dict(max_iter=max_iter, tol=tol, trace=unrolled)
    nom = forward(*(inst[k] for k in KEYS), **kw)
    plus = forward(*(_perturbed(inst, key, E, +eps)[k] for k in KEYS), **kw)
    minus = forward(*(_perturbed(inst, key, E, -eps)[k] for k in KEYS), **kw)
    s0 = _signature(nom, unrolled)
    valid = _signature(plus, unrolled) == s0 and _signature(minus, unrolled) == s0
    if not unrolled:
        valid = valid and nom["status"] == ST_CONVERGED
    d = float(np.dot(abar, (plus["a"] - minus["a"]) / (2.0 * eps)))
    return d, valid


def random_direction(rng, x, symmetric=False):
    """Random perturbation direction scaled to the magnitude of input ``x``.

    Entries are ``N(0,1) * (|x| + 1e-3 max|x|)`` so that inputs spanning
    orders of magnitude (D runs from 1e2 to 1e4) get a relative perturbation;
    ``symmetric`` keeps a mass-matrix perturbation symmetric.
    """
    x = np.asarray(x, dtype=np.float64)
    mag = np.abs(x) + 1e-3 * (np.abs(x).max() if x.size else 0.0) + 1e-300
    E = rng.standard_normal(x.shape) * mag
    if symmetric:
        E = 0.5 * (E + E.T)
    return E
