"""FP64 CPU oracle for the batched regularised contact solve (test infrastructure).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It never imports the GPU package and the
GPU package never imports it; the two meet only through the seeded input
generator.

``oracle.c`` (compiled to ``liboracle.so`` by :func:`build`) holds the
method: Newton steps with QR solves and an exact sort-and-scan line search
(Sec. III-B, eqs. 6, 9, 10), the IFT adjoint VJP (Sec. III-C, eq. 17) and
the unrolled-trace VJP, the IFT Jacobian-vector products (eq. 15, forward
mode), and a nonlinear conjugate-gradient forward solve for the same
minimiser.  ``brute.py`` pins the forward result by active-set
enumeration; ``fd.py`` pins the gradients by central finite differences.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

ST_CONVERGED, ST_MAXITER, ST_NONFINITE, ST_NOTSPD = 1, 2, 4, 8


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc (plain -O2, OpenMP across instances)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_i32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


class _Opt:
    """ndpointer argtype that also accepts None (NULL)."""

    def __init__(self, base):
        self.base = base

    def from_param(self, obj):
        if obj is None:
            return None
        return self.base.from_param(obj)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        i, d = C.c_int, C.c_double
        L.oracle_forward.argtypes = [i, i, _dp, _dp, _dp, _dp, _dp, _Opt(_dp), i, d, _dp, _u8,
                                     C.POINTER(i), C.POINTER(i), _Opt(_dp), _Opt(_u8), _Opt(_u8)]
        L.oracle_ift_vjp.argtypes = [i, i, _dp, _dp, _dp, _dp, _dp, _dp, _Opt(_u8), _dp,
                                     _Opt(_dp), _Opt(_dp), _Opt(_dp), _Opt(_dp), _Opt(_dp),
                                     _Opt(_dp)]
        L.oracle_unrolled_vjp.argtypes = [i, i, _dp, _dp, _dp, _dp, _dp, _dp, i, d, _dp,
                                          _Opt(_dp), _Opt(_dp), _Opt(_dp), _Opt(_dp), _Opt(_dp),
                                          C.POINTER(i), C.POINTER(i)]
        L.oracle_ift_jvp.argtypes = [i, i, _dp, _dp, _dp, _u8, i, _Opt(_dp), _Opt(_dp), _dp]
        L.oracle_line_search.argtypes = [i, i, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _u8]
        L.oracle_line_search.restype = C.c_double
        L.oracle_max_threads.restype = C.c_int
        pk = [i, _i32, _i32, _i64, _i64, _i64, _i64]
        L.oracle_forward_batch.argtypes = pk + [_dp, _dp, _dp, _dp, _dp, i, d, _dp, _u8, _i32,
                                                _i32, i]
        L.oracle_ift_vjp_batch.argtypes = pk + [_dp, _dp, _dp, _dp, _dp, _dp, _Opt(_u8), _dp,
                                                _Opt(_dp), _Opt(_dp), _Opt(_dp), _Opt(_dp),
                                                _Opt(_dp), i]
        L.oracle_ift_jvp_batch.argtypes = pk + [_dp, _dp, _dp, _u8, i, _Opt(_dp), _Opt(_dp), _dp, i]
        L.oracle_ell_block.argtypes = [_dp, d, d, d, _dp, _dp, C.POINTER(d)]
        L.oracle_ell_block.restype = i
        L.oracle_ell_objective.argtypes = [i, i, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.oracle_ell_objective.restype = d
        L.oracle_forward_ell.argtypes = [i, i, _dp, _dp, _dp, _dp, _dp, _dp, _dp, i, d, _dp, _u8,
                                         C.POINTER(i), C.POINTER(i)]
        L.oracle_ift_vjp_ell.argtypes = [i, i] + [_dp] * 16
        L.oracle_forward_rows.argtypes = [i, i, _dp, _dp, _dp, _dp, _dp, _u8, _dp, i, d, _dp, _u8,
                                          C.POINTER(i), C.POINTER(i)]
        L.oracle_ift_vjp_rows.argtypes = [i, i, _dp, _dp, _dp, _dp, _dp, _u8, _dp, _dp, _dp] + \
            [_dp] * 6
        L.oracle_forward_cg.argtypes = [i, i, _dp, _dp, _dp, _dp, _dp, i, d, _dp, _u8,
                                        C.POINTER(i), C.POINTER(i)]
        L.oracle_forward_cg_batch.argtypes = pk + [_dp, _dp, _dp, _dp, _dp, i, d, _dp, _u8, _i32,
                                                   _i32, i]
        L.oracle_unrolled_vjp_batch.argtypes = pk + [_dp, _dp, _dp, _dp, _dp, _dp, i, d, _dp,
                                                     _Opt(_dp), _Opt(_dp), _Opt(_dp), _Opt(_dp),
                                                     _Opt(_dp), _i32, _i32, i]
        _lib = L
    return _lib


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def max_threads() -> int:
    return int(lib().oracle_max_threads())


# ---------------------------------------------------------------- one instance

def forward(M, J, a0, aref, D, a_init=None, max_iter=10, tol=1e-10, trace=False):
    """Solve one instance.  Returns dict(a, active, iters, status[, alphas, A, Ap])."""
    M, J, a0, aref, D = map(_f64, (M, J, a0, aref, D))
    n = a0.shape[0]
    m = aref.shape[0]
    J = J.reshape(m, n)
    a = np.empty(n)
    act = np.empty(m, dtype=np.uint8)
    it, st = C.c_int(0), C.c_int(0)
    K = max(max_iter, 0)
    al = np.zeros(max(K, 1)) if trace else None
    tA = np.zeros((max(K, 1), max(m, 1)), dtype=np.uint8) if trace else None
    tAp = np.zeros((max(K, 1), max(m, 1)), dtype=np.uint8) if trace else None
    lib().oracle_forward(n, m, M, J, a0, aref, D, None if a_init is None else _f64(a_init),
                         max_iter, tol, a, act, C.byref(it), C.byref(st), al, tA, tAp)
    out = dict(a=a, active=act.astype(bool), iters=it.value, status=st.value)
    if trace:
        k = it.value
        out.update(alphas=al[:k], A=tA[:k, :m].astype(bool), Ap=tAp[:k, :m].astype(bool))
    return out


def forward_cg(M, J, a0, aref, D, max_iter=200, tol=1e-10):
    """Solve one instance by preconditioned nonlinear CG with the exact line
    search.  Returns dict(a, active, iters, status)."""
    M, J, a0, aref, D = map(_f64, (M, J, a0, aref, D))
    n, m = a0.shape[0], aref.shape[0]
    J = J.reshape(m, n)
    a = np.empty(n)
    act = np.empty(max(m, 1), dtype=np.uint8)
    it, st = C.c_int(0), C.c_int(0)
    lib().oracle_forward_cg(n, m, M, J, a0, aref, D, max_iter, tol, a, act, C.byref(it),
                            C.byref(st))
    return dict(a=a, active=act[:m].astype(bool), iters=it.value, status=st.value)


def ell_block(u, dn, dt, mu):
    """One contact of the round cone at u (3): (zone, w = ds/du, G = d2s/du2, s)."""
    u = _f64(u)
    w = np.empty(3)
    G = np.empty(9)
    sv = C.c_double(0.0)
    z = lib().oracle_ell_block(u, float(dn), float(dt), float(mu), w, G, C.byref(sv))
    return z, w, G.reshape(3, 3), sv.value


def ell_objective(M, J, a0, aref, dn, dt, mu, a):
    """L(a) and F(a) with the round cone."""
    M, J, a0, aref, dn, dt, mu, a = map(_f64, (M, J, a0, aref, dn, dt, mu, a))
    n, nc = a0.shape[0], dn.shape[0]
    F = np.empty(n)
    Lv = lib().oracle_ell_objective(n, nc, M, J.reshape(3 * nc, n), a0, aref, dn, dt, mu, a, F)
    return Lv, F


def forward_ell(M, J, a0, aref, dn, dt, mu, max_iter=60, tol=1e-12):
    """Round-cone forward solve.  Returns dict(a, zone, iters, status)."""
    M, J, a0, aref, dn, dt, mu = map(_f64, (M, J, a0, aref, dn, dt, mu))
    n, nc = a0.shape[0], dn.shape[0]
    a = np.empty(n)
    zone = np.empty(max(nc, 1), dtype=np.uint8)
    it, st = C.c_int(0), C.c_int(0)
    lib().oracle_forward_ell(n, nc, M, J.reshape(3 * nc, n), a0, aref, dn, dt, mu, max_iter, tol,
                             a, zone, C.byref(it), C.byref(st))
    return dict(a=a, zone=zone[:nc].copy(), iters=it.value, status=st.value)


def ift_vjp_ell(M, J, a0, aref, dn, dt, mu, a, abar):
    """Round-cone IFT VJP at a.  Returns dict(a0, aref, J, dn, dt, mu, M)."""
    M, J, a0, aref, dn, dt, mu, a, abar = map(_f64, (M, J, a0, aref, dn, dt, mu, a, abar))
    n, nc = a0.shape[0], dn.shape[0]
    m = 3 * nc
    out = dict(a0=np.empty(n), aref=np.empty(max(m, 1)), J=np.empty(max(m * n, 1)),
               dn=np.empty(max(nc, 1)), dt=np.empty(max(nc, 1)), mu=np.empty(max(nc, 1)),
               M=np.empty(n * n))
    lib().oracle_ift_vjp_ell(n, nc, M, J.reshape(m, n), a0, aref, dn, dt, mu, a, abar, out["a0"],
                             out["aref"], out["J"], out["dn"], out["dt"], out["mu"], out["M"])
    out["aref"] = out["aref"][:m]
    out["J"] = out["J"][:m * n].reshape(m, n)
    out["M"] = out["M"].reshape(n, n)
    for k in ("dn", "dt", "mu"):
        out[k] = out[k][:nc]
    return out


def forward_rows(M, J, a0, aref, D, kind, floss, max_iter=60, tol=1e-12):
    """Mixed rows (kind 0 one-sided, 1 equality, 2 friction loss with bound floss).
    Returns dict(a, zone, iters, status); zone per row: 0 no force, 1 quadratic,
    2 / 3 saturated at +f / -f."""
    M, J, a0, aref, D, floss = map(_f64, (M, J, a0, aref, D, floss))
    kind = np.ascontiguousarray(kind, dtype=np.uint8)
    n, m = a0.shape[0], aref.shape[0]
    a = np.empty(n)
    zone = np.empty(max(m, 1), dtype=np.uint8)
    it, st = C.c_int(0), C.c_int(0)
    lib().oracle_forward_rows(n, m, M, J.reshape(m, n) if m else np.zeros((1, n)), a0, aref, D,
                              kind if m else np.zeros(1, np.uint8), floss, max_iter, tol, a, zone,
                              C.byref(it), C.byref(st))
    return dict(a=a, zone=zone[:m].copy(), iters=it.value, status=st.value)


def ift_vjp_rows(M, J, a0, aref, D, kind, floss, a, abar):
    """Mixed-row IFT VJP at a.  Returns dict(a0, aref, J, D, floss, M)."""
    M, J, a0, aref, D, floss, a, abar = map(_f64, (M, J, a0, aref, D, floss, a, abar))
    kind = np.ascontiguousarray(kind, dtype=np.uint8)
    n, m = a0.shape[0], aref.shape[0]
    out = dict(a0=np.empty(n), aref=np.empty(max(m, 1)), J=np.empty(max(m * n, 1)),
               D=np.empty(max(m, 1)), floss=np.empty(max(m, 1)), M=np.empty(n * n))
    lib().oracle_ift_vjp_rows(n, m, M, J.reshape(m, n), a0, aref, D, kind, floss, a, abar,
                              out["a0"], out["aref"], out["J"], out["D"], out["floss"], out["M"])
    out["J"] = out["J"][:m * n].reshape(m, n)
    out["M"] = out["M"].reshape(n, n)
    for k in ("aref", "D", "floss"):
        out[k] = out[k][:m]
    return out


def ift_vjp(M, J, a0, aref, D, a, abar, active=None):
    """IFT VJP at solution ``a`` (eq. 17).  Returns dict of the five cotangents + lambda."""
    M, J, a0, aref, D, a, abar = map(_f64, (M, J, a0, aref, D, a, abar))
    n, m = a0.shape[0], aref.shape[0]
    J = J.reshape(m, n)
    out = dict(a0=np.empty(n), aref=np.empty(m), J=np.empty((m, n)), D=np.empty(m),
               M=np.empty((n, n)), lam=np.empty(n))
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    lib().oracle_ift_vjp(n, m, M, J, a0, aref, D, a, act, abar, out["a0"], out["aref"],
                         out["J"], out["D"], out["M"], out["lam"])
    return out


def ift_jvp(M, J, D, active, da0=None, daref=None, k=None):
    """IFT Jacobian-vector products (eq. 15) for k directions of (a0, aref):
    da0 [k, n] and daref [k, m] (either None for zero).  Returns da [k, n]."""
    M, J, D = map(_f64, (M, J, D))
    n, m = M.shape[0], D.shape[0]
    J = J.reshape(m, n)
    if k is None:
        k = (da0 if da0 is not None else daref).shape[0]
    act = np.ascontiguousarray(active, dtype=np.uint8)
    d0 = None if da0 is None else _f64(da0).reshape(k, n)
    dr = None if daref is None else _f64(daref).reshape(k, m)
    da = np.empty((max(k, 1), max(n, 1)))
    lib().oracle_ift_jvp(n, m, M, J, D, act if m else np.zeros(1, np.uint8), k, d0, dr, da)
    return da[:k, :n]


def unrolled_vjp(M, J, a0, aref, D, abar, K, tol=1e-10):
    """Gradient of abar . a_K through the executed K-step trace."""
    M, J, a0, aref, D, abar = map(_f64, (M, J, a0, aref, D, abar))
    n, m = a0.shape[0], aref.shape[0]
    J = J.reshape(m, n)
    out = dict(a=np.empty(n), a0=np.empty(n), aref=np.empty(m), J=np.empty((m, n)),
               D=np.empty(m), M=np.empty((n, n)))
    it, st = C.c_int(0), C.c_int(0)
    lib().oracle_unrolled_vjp(n, m, M, J, a0, aref, D, abar, K, tol, out["a"], out["a0"],
                              out["aref"], out["J"], out["D"], out["M"], C.byref(it),
                              C.byref(st))
    out.update(iters=it.value, status=st.value)
    return out


def line_search(M, J, a0, aref, D, a, p):
    """Exact line search alone.  Returns (alpha, Ap, q)."""
    M, J, a0, aref, D, a, p = map(_f64, (M, J, a0, aref, D, a, p))
    n, m = a0.shape[0], aref.shape[0]
    J = J.reshape(m, n)
    q = np.empty(max(m, 1))
    Ap = np.empty(max(m, 1), dtype=np.uint8)
    alpha = lib().oracle_line_search(n, m, M, J, a0, aref, D, a, p, q, Ap)
    return alpha, Ap[:m].astype(bool), q[:m]


# ---------------------------------------------------------------- batches

class Packed:
    """Packed batch description (flat FP64 arrays + element offsets)."""

    def __init__(self, nv, nrows, M, J, a0, aref, D, abar=None):
        self.nv = np.ascontiguousarray(nv, dtype=np.int32)
        self.nrows = np.ascontiguousarray(nrows, dtype=np.int32)
        nv64, nr64 = self.nv.astype(np.int64), self.nrows.astype(np.int64)
        cs = lambda s: np.concatenate([[0], np.cumsum(s)]).astype(np.int64)
        self.off_nn, self.off_mn = cs(nv64 * nv64), cs(nv64 * nr64)
        self.off_n, self.off_m = cs(nv64), cs(nr64)
        self.M, self.J, self.a0, self.aref, self.D = (_f64(x).ravel() for x in (M, J, a0, aref, D))
        self.abar = None if abar is None else _f64(abar).ravel()
        self.B = int(self.nv.shape[0])

    @classmethod
    def uniform(cls, M, J, a0, aref, D, abar=None):
        B, m, n = J.shape
        return cls(np.full(B, n), np.full(B, m), M, J, a0, aref, D, abar)

    def _pk(self):
        return (self.B, self.nv, self.nrows, self.off_nn, self.off_mn, self.off_n, self.off_m)

    def _buf(self, key):
        size = {"n": self.off_n[-1], "m": self.off_m[-1], "mn": self.off_mn[-1],
                "nn": self.off_nn[-1]}[key]
        return np.zeros(max(int(size), 1))

    def forward(self, max_iter=10, tol=1e-10, threads=0):
        a = self._buf("n")
        act = np.zeros(max(int(self.off_m[-1]), 1), dtype=np.uint8)
        it = np.zeros(self.B, dtype=np.int32)
        st = np.zeros(self.B, dtype=np.int32)
        lib().oracle_forward_batch(*self._pk(), self.M, self.J, self.a0, self.aref, self.D,
                                   max_iter, tol, a, act, it, st, threads)
        return dict(a=a, active=act, iters=it, status=st)

    def forward_cg(self, max_iter=200, tol=1e-10, threads=0):
        a = self._buf("n")
        act = np.zeros(max(int(self.off_m[-1]), 1), dtype=np.uint8)
        it = np.zeros(self.B, dtype=np.int32)
        st = np.zeros(self.B, dtype=np.int32)
        lib().oracle_forward_cg_batch(*self._pk(), self.M, self.J, self.a0, self.aref, self.D,
                                      max_iter, tol, a, act, it, st, threads)
        return dict(a=a, active=act, iters=it, status=st)

    def ift_vjp(self, a, active, abar=None, threads=0, outputs=("a0", "aref", "J", "D", "M")):
        abar = self.abar if abar is None else _f64(abar).ravel()
        g = {k: (self._buf({"a0": "n", "aref": "m", "J": "mn", "D": "m", "M": "nn"}[k])
                 if k in outputs else None) for k in ("a0", "aref", "J", "D", "M")}
        lib().oracle_ift_vjp_batch(*self._pk(), self.M, self.J, self.a0, self.aref, self.D,
                                   _f64(a).ravel(),
                                   None if active is None else np.ascontiguousarray(active, np.uint8),
                                   abar, g["a0"], g["aref"], g["J"], g["D"], g["M"], threads)
        return g

    def ift_jvp(self, active, k, da0=None, daref=None, threads=0):
        """Directional derivatives of a* for k directions per instance:
        da0 [k * total_n] (instance i at k * off_n[i], direction-major) and
        daref [k * total_m] (at k * off_m[i]), either None.  Returns da
        [k * total_n]."""
        da = np.zeros(max(k * int(self.off_n[-1]), 1))
        act = np.ascontiguousarray(active, dtype=np.uint8)
        if act.size == 0:
            act = np.zeros(1, np.uint8)
        lib().oracle_ift_jvp_batch(*self._pk(), self.M, self.J, self.D, act, k,
                                   None if da0 is None else _f64(da0).ravel(),
                                   None if daref is None else _f64(daref).ravel(), da, threads)
        return da

    def unrolled_vjp(self, K, tol=1e-10, abar=None, threads=0):
        abar = self.abar if abar is None else _f64(abar).ravel()
        a = self._buf("n")
        g = dict(a0=self._buf("n"), aref=self._buf("m"), J=self._buf("mn"), D=self._buf("m"),
                 M=self._buf("nn"))
        it = np.zeros(self.B, dtype=np.int32)
        st = np.zeros(self.B, dtype=np.int32)
        lib().oracle_unrolled_vjp_batch(*self._pk(), self.M, self.J, self.a0, self.aref, self.D,
                                        abar, K, tol, a, g["a0"], g["aref"], g["J"], g["D"],
                                        g["M"], it, st, threads)
        g.update(a=a, iters=it, status=st)
        return g
