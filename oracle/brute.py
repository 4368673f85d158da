"""Brute-force active-set enumeration (test infrastructure; NumPy, FP64).

Independent of ``oracle.c``: it does not iterate at all.  For a strictly
convex piecewise quadratic (Sec. III-A, eq. 5 with pyramidal rows) the
minimiser ``a*`` is the unique point where the stationarity residual
(eq. 6) vanishes.  For every subset ``S`` of rows the quadratic obtained by
declaring exactly ``S`` active has the minimiser

    (M + J_S^T diag(D_S) J_S) a_S = M a0 + J_S^T diag(D_S) aref_S,

and ``S`` is *consistent* when ``r_i(a_S) < 0`` exactly for ``i`` in ``S``.  A
consistent ``S`` makes ``F(a_S) = 0``, so ``a_S = a*`` by uniqueness, and
``S = A(a*)`` is always consistent.  Subsets that are consistent only within
a band ``|r_i| <= band`` mark the instance as degenerate.
"""
from __future__ import annotations

import numpy as np


def all_masks(m: int) -> np.ndarray:
    """[2^m, m] boolean matrix of every subset of ``m`` rows."""
    idx = np.arange(1 << m, dtype=np.int64)
    return ((idx[:, None] >> np.arange(m)[None, :]) & 1).astype(bool)


def enumerate_solutions(M, J, a0, aref, D, band: float = 0.0, chunk: int = 1 << 14):
    """Return (a_star, S_star, n_consistent, n_band).

    ``a_star``/``S_star`` come from the consistent subset (strict rule);
    ``n_band`` counts subsets consistent within ``band``.
    """
    M, J, a0, aref, D = (np.asarray(x, dtype=np.float64) for x in (M, J, a0, aref, D))
    m, n = J.shape
    if m > 20:
        raise ValueError("brute force limited to m <= 20 rows")
    Ma0 = M @ a0
    best = None
    n_cons = 0
    n_band = 0
    total = 1 << m
    for start in range(0, total, chunk):
        idx = np.arange(start, min(total, start + chunk), dtype=np.int64)
        S = ((idx[:, None] >> np.arange(m)[None, :]) & 1).astype(np.float64)   # [s, m]
        W = S * D[None, :]                                                      # D_S
        H = M[None] + np.einsum("ri,sr,rj->sij", J, W, J)
        rhs = Ma0[None] + np.einsum("ri,sr->si", J, W * aref[None, :])
        aS = np.linalg.solve(H, rhs[..., None])[..., 0]                         # [s, n]
        r = aS @ J.T - aref[None, :]                                            # [s, m]
        Sb = S.astype(bool)
        strict = np.all((r < 0) == Sb, axis=1)
        loose = np.all(np.where(Sb, r < band, r > -band), axis=1)
        n_cons += int(strict.sum())
        n_band += int(loose.sum())
        if best is None and strict.any():
            k = int(np.flatnonzero(strict)[0])
            best = (aS[k].copy(), Sb[k].copy())
    if best is None:
        return None, None, 0, n_band
    return best[0], best[1], n_cons, n_band
