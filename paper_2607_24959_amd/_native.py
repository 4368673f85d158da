"""ctypes binding of libcs.so: the C ABI of include/cs.h and include/cs_serve.h.

Every function here marshals arguments and calls the library; all of the
method runs in the HIP kernels.  Importing this module loads the library and
raises if it has not been built -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcs.so")

CS_OK, CS_EINVAL, CS_ENOSPC, CS_EHIP, CS_EUNSUPPORTED = 0, -1, -2, -3, -4
CS_F32, CS_F64 = 0, 1
ST_CONVERGED, ST_MAXITER, ST_NONFINITE, ST_NOTSPD, ST_LSFAIL, ST_BADDESC = 1, 2, 4, 8, 16, 32
NV_MAX, NROWS_MAX = 128, 4096
STATIC_TAPE_BYTES = 64 << 20
PATH_AUTO, PATH_TEAM, PATH_SMALL, PATH_CHUNK, PATH_WAVE = 0, 1, 2, 3, 4
UNROLLED_RECORD, UNROLLED_REPLAY, FORWARD_CG = 1, 2, 4
ROLLOUT_FORWARD, ROLLOUT_BACKWARD, ROLLOUT_RECOMPUTE = 1, 2, 4

EXPORTED = ("cs_forward", "cs_ift_vjp", "cs_ift_jvp", "cs_unrolled_vjp", "cs_unrolled_vjp_static",
            "cs_rollout", "cs_rollout_workspace_bytes", "cs_forward_ell", "cs_ift_vjp_ell",
            "cs_forward_rows", "cs_ift_vjp_rows",
            "cs_state_bytes",
            "cs_unrolled_tape_bytes", "cs_strerror", "cs_version",
            "cs_serve_admit", "cs_serve_pre", "cs_serve_post", "cs_serve_tick")


class CsBatch(C.Structure):
    _fields_ = [
        ("B", C.c_int32), ("dtype", C.c_int32),
        ("nv_uniform", C.c_int32), ("nrows_uniform", C.c_int32),
        ("nv", C.c_void_p), ("nrows", C.c_void_p),
        ("off_nn", C.c_void_p), ("off_mn", C.c_void_p),
        ("off_n", C.c_void_p), ("off_m", C.c_void_p),
        ("order", C.c_void_p),
        ("nv_max", C.c_int32), ("nrows_max", C.c_int32),
        ("total_nn", C.c_int64), ("total_mn", C.c_int64),
        ("total_n", C.c_int64), ("total_m", C.c_int64),
        ("path", C.c_int32), ("count", C.c_int32),
    ]


class CsSolverParams(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("flags", C.c_int32), ("tol", C.c_double)]


class CsRolloutParams(C.Structure):
    _fields_ = [("horizon", C.c_int32), ("flags", C.c_int32), ("max_iter", C.c_int32),
                ("reserved", C.c_int32), ("tol", C.c_double), ("h", C.c_double),
                ("b_damp", C.c_double)]


class CsServeTable(C.Structure):
    _fields_ = [
        ("dtype", C.c_int32), ("slots", C.c_int32), ("window", C.c_int32),
        ("n_cap", C.c_int32), ("m_cap", C.c_int32), ("reserved", C.c_int32),
        ("h", C.c_double), ("b_damp", C.c_double), ("k_spring", C.c_double),
        ("M", C.c_void_p), ("Minv", C.c_void_p), ("J", C.c_void_p), ("D", C.c_void_p),
        ("pen", C.c_void_p), ("v", C.c_void_p), ("goal", C.c_void_p), ("tau", C.c_void_p),
        ("nv", C.c_void_p), ("nrows", C.c_void_p),
        ("vbar", C.c_void_p), ("taubar", C.c_void_p),
        ("a0", C.c_void_p), ("abar", C.c_void_p), ("a", C.c_void_p), ("a0bar", C.c_void_p),
        ("aref", C.c_void_p), ("arefbar", C.c_void_p),
        ("state", C.c_void_p), ("mask_offset", C.c_uint64),
        ("arch_a", C.c_void_p), ("arch_a0", C.c_void_p), ("arch_aref", C.c_void_p),
        ("arch_fac", C.c_void_p), ("arch_mask", C.c_void_p),
    ]


class CsError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {strerror(code)} ({code})")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libcs.so is not built ({LIB_PATH}); run "
                              "paper_2607_24959_amd.build.build() first")
        L = C.CDLL(LIB_PATH)
        vp, sz, i32 = C.c_void_p, C.c_size_t, C.c_int32
        pb, pp = C.POINTER(CsBatch), C.POINTER(CsSolverParams)
        L.cs_version.restype = C.c_int
        L.cs_strerror.restype = C.c_char_p
        L.cs_strerror.argtypes = [C.c_int]
        L.cs_state_bytes.restype = sz
        L.cs_state_bytes.argtypes = [pb]
        L.cs_unrolled_tape_bytes.restype = sz
        L.cs_unrolled_tape_bytes.argtypes = [pb, i32]
        L.cs_forward.restype = C.c_int
        L.cs_forward.argtypes = [pb, pp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp, vp, vp]
        L.cs_ift_vjp.restype = C.c_int
        L.cs_ift_vjp.argtypes = [pb, vp, sz, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.cs_ift_jvp.restype = C.c_int
        L.cs_ift_jvp.argtypes = [pb, vp, sz, vp, vp, vp, i32, vp, vp, vp, vp]
        L.cs_forward_ell.restype = C.c_int
        L.cs_forward_ell.argtypes = [pb, pp] + [vp] * 10 + [sz, vp, vp, vp]
        L.cs_ift_vjp_ell.restype = C.c_int
        L.cs_ift_vjp_ell.argtypes = [pb, vp, sz] + [vp] * 17
        L.cs_forward_rows.restype = C.c_int
        L.cs_forward_rows.argtypes = [pb, pp] + [vp] * 10 + [sz, vp, vp, vp]
        L.cs_ift_vjp_rows.restype = C.c_int
        L.cs_ift_vjp_rows.argtypes = [pb, vp, sz] + [vp] * 16
        prp = C.POINTER(CsRolloutParams)
        L.cs_rollout_workspace_bytes.restype = sz
        L.cs_rollout_workspace_bytes.argtypes = [pb, prp]
        L.cs_rollout.restype = C.c_int
        L.cs_rollout.argtypes = [pb, prp] + [vp] * 12 + [sz, vp, vp, vp]
        L.cs_unrolled_vjp.restype = C.c_int
        L.cs_unrolled_vjp.argtypes = [pb, pp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                      sz, vp, vp, vp]
        L.cs_unrolled_vjp_static.restype = C.c_int
        L.cs_unrolled_vjp_static.argtypes = [pb, pp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                             vp, vp, vp, vp]
        pt = C.POINTER(CsServeTable)
        L.cs_serve_admit.restype = C.c_int
        L.cs_serve_admit.argtypes = [pt, pt, vp, i32, vp]
        for name in ("cs_serve_pre", "cs_serve_post"):
            getattr(L, name).restype = C.c_int
            getattr(L, name).argtypes = [pt, vp, i32, vp]
        L.cs_serve_tick.restype = C.c_int
        L.cs_serve_tick.argtypes = [pt, pt, pb, i32, pp, sz, vp, vp, vp, vp, i32, i32, i32, vp, i32,
                                    vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().cs_strerror(int(code)).decode()


def check(code: int, where: str) -> None:
    if code != CS_OK:
        raise CsError(code, where)


def version() -> int:
    return int(lib().cs_version())


def state_bytes(batch: CsBatch) -> int:
    return int(lib().cs_state_bytes(C.byref(batch)))


def tape_bytes(batch: CsBatch, K: int) -> int:
    return int(lib().cs_unrolled_tape_bytes(C.byref(batch), int(K)))


def forward(batch, params, M, J, a0, aref, D, a_init, a_out, state, state_nbytes, status, iters,
            stream):
    return lib().cs_forward(C.byref(batch), C.byref(params), M, J, a0, aref, D, a_init, a_out,
                            state, state_nbytes, status, iters, stream)


def ift_vjp(batch, state, state_nbytes, M, J, a0, aref, D, a, abar, a0bar, arefbar, Jbar, Dbar,
            Mbar, stream):
    return lib().cs_ift_vjp(C.byref(batch), state, state_nbytes, M, J, a0, aref, D, a, abar,
                            a0bar, arefbar, Jbar, Dbar, Mbar, stream)


def ift_jvp(batch, state, state_nbytes, M, J, D, k, da0, daref, da, stream):
    return lib().cs_ift_jvp(C.byref(batch), state, state_nbytes, M, J, D, int(k), da0, daref, da,
                            stream)


def forward_ell(batch, params, M, J, a0, aref, dn, dt, mu, a_init, a_out, state, state_nbytes,
                status, iters, stream):
    return lib().cs_forward_ell(C.byref(batch), C.byref(params), M, J, a0, aref, dn, dt, mu, a_init,
                                a_out, state, state_nbytes, status, iters, stream)


def ift_vjp_ell(batch, state, state_nbytes, M, J, a0, aref, dn, dt, mu, a, abar, a0bar, arefbar,
                Jbar, dnbar, dtbar, mubar, Mbar, stream):
    return lib().cs_ift_vjp_ell(C.byref(batch), state, state_nbytes, M, J, a0, aref, dn, dt, mu, a,
                                abar, a0bar, arefbar, Jbar, dnbar, dtbar, mubar, Mbar, stream)


def forward_rows(batch, params, M, J, a0, aref, D, kind, floss, a_init, a_out, state, state_nbytes,
                 status, iters, stream):
    return lib().cs_forward_rows(C.byref(batch), C.byref(params), M, J, a0, aref, D, kind, floss,
                                 a_init, a_out, state, state_nbytes, status, iters, stream)


def ift_vjp_rows(batch, state, state_nbytes, M, J, a0, aref, D, kind, floss, a, abar, a0bar,
                 arefbar, Jbar, Dbar, flossbar, Mbar, stream):
    return lib().cs_ift_vjp_rows(C.byref(batch), state, state_nbytes, M, J, a0, aref, D, kind, floss,
                                 a, abar, a0bar, arefbar, Jbar, Dbar, flossbar, Mbar, stream)


def rollout_workspace_bytes(batch, params):
    return lib().cs_rollout_workspace_bytes(C.byref(batch), C.byref(params))


def rollout(batch, params, M, J, D, c, v0, tau, v_goal, vbar_T, v_T, tau_bar, v0_bar, ws, ws_nbytes,
            status, iters, stream):
    return lib().cs_rollout(C.byref(batch), C.byref(params), M, J, D, c, v0, tau, v_goal, vbar_T,
                            v_T, tau_bar, v0_bar, ws, ws_nbytes, status, iters, stream)


def unrolled_vjp(batch, params, M, J, a0, aref, D, abar, a_out, a0bar, arefbar, Jbar, Dbar, Mbar,
                 tape, tape_nbytes, status, iters, stream):
    return lib().cs_unrolled_vjp(C.byref(batch), C.byref(params), M, J, a0, aref, D, abar, a_out,
                                 a0bar, arefbar, Jbar, Dbar, Mbar, tape, tape_nbytes, status,
                                 iters, stream)


def unrolled_vjp_static(batch, params, M, J, a0, aref, D, abar, a_out, a0bar, arefbar, Jbar,
                        Dbar, Mbar, status, iters, stream):
    """cs_unrolled_vjp_static: the unrolled VJP with the library's static tape."""
    return lib().cs_unrolled_vjp_static(C.byref(batch), C.byref(params), M, J, a0, aref, D, abar,
                                        a_out, a0bar, arefbar, Jbar, Dbar, Mbar, status, iters,
                                        stream)


def serve_admit(table, pool, pairs, count, stream):
    return lib().cs_serve_admit(C.byref(table), C.byref(pool), pairs, int(count), stream)


def serve_pre(table, entries, count, stream):
    return lib().cs_serve_pre(C.byref(table), entries, int(count), stream)


def serve_post(table, entries, count, stream):
    return lib().cs_serve_post(C.byref(table), entries, int(count), stream)


def serve_tick(table, pool, classes, nclasses, params, state_nbytes, status, iters, host_list,
               dev_list, list_len, n_admit, n_entries, launches, nlaunch, stream, side, ev_list,
               ev_fork, ev_join):
    """One serving tick's device work (list upload, admit, pre, the solver
    launches on two lanes, post); ``classes`` is a ctypes array of CsBatch and
    ``launches`` the address of an int32 [nlaunch, 5] array of
    (kind, class, lane, count, order) rows."""
    return lib().cs_serve_tick(C.byref(table), None if pool is None else C.byref(pool), classes,
                               int(nclasses), C.byref(params), state_nbytes, status, iters,
                               host_list, dev_list, int(list_len), int(n_admit), int(n_entries),
                               launches, int(nlaunch), stream, side, ev_list, ev_fork, ev_join)
