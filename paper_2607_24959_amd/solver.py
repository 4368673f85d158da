"""Torch-facing wrappers of the C ABI (device memory and streams only).

PyTorch supplies device allocations and the current HIP stream; every step
of the method runs inside libcs.so.  Shapes are checked here on the host
against the batch descriptor before any pointer reaches a kernel.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _native as N

_DT = {torch.float32: N.CS_F32, torch.float64: N.CS_F64}


def _vp(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Batch:
    """A batch descriptor (uniform or packed) plus the device arrays behind it.

    Sizes of every per-instance array are known on the host: ``total_n``
    elements for n-vectors, ``total_m`` for row vectors, ``total_mn`` for J,
    ``total_nn`` for M.
    """

    def __init__(self, B, dtype, device, n=None, m=None, nv=None, nrows=None, order=None,
                 path=N.PATH_AUTO):
        self.B = int(B)
        self.dtype = dtype
        self.device = torch.device(device)
        if dtype not in _DT:
            raise ValueError(f"unsupported dtype {dtype}")
        d = N.CsBatch()
        d.B = self.B
        d.dtype = _DT[dtype]
        self._keep = []
        if nv is None:
            self.packed = False
            self.n, self.m = int(n), int(m)
            d.nv_uniform, d.nrows_uniform = self.n, self.m
            self.nv_host = np.full(self.B, self.n, dtype=np.int32)
            self.nrows_host = np.full(self.B, self.m, dtype=np.int32)
        else:
            self.packed = True
            self.nv_host = np.ascontiguousarray(nv, dtype=np.int32)
            self.nrows_host = np.ascontiguousarray(nrows, dtype=np.int32)
            if self.nv_host.shape != (self.B,) or self.nrows_host.shape != (self.B,):
                raise ValueError("nv / nrows must have shape [B]")
            if self.B and (self.nv_host.min() < 1 or self.nrows_host.min() < 0):
                raise ValueError("need n >= 1 and m >= 0 for every instance")
        nv64 = self.nv_host.astype(np.int64)
        nr64 = self.nrows_host.astype(np.int64)
        off = lambda s: np.concatenate([[0], np.cumsum(s)]).astype(np.int64)
        self.off_nn, self.off_mn = off(nv64 * nv64), off(nv64 * nr64)
        self.off_n, self.off_m = off(nv64), off(nr64)
        self.total_nn, self.total_mn = int(self.off_nn[-1]), int(self.off_mn[-1])
        self.total_n, self.total_m = int(self.off_n[-1]), int(self.off_m[-1])
        self.nv_max = int(self.nv_host.max()) if self.B else 1
        self.nrows_max = int(self.nrows_host.max()) if self.B else 0
        if self.packed:
            dev = lambda x: self._dev(torch.from_numpy(np.ascontiguousarray(x)))
            d.nv, d.nrows = dev(self.nv_host), dev(self.nrows_host)
            d.off_nn, d.off_mn = dev(self.off_nn), dev(self.off_mn)
            d.off_n, d.off_m = dev(self.off_n), dev(self.off_m)
            d.nv_max, d.nrows_max = self.nv_max, self.nrows_max
            d.total_nn, d.total_mn = self.total_nn, self.total_mn
            d.total_n, d.total_m = self.total_n, self.total_m
        if order is not None:
            order = np.ascontiguousarray(order, dtype=np.int32)
            if order.shape != (self.B,) or not np.array_equal(np.sort(order), np.arange(self.B)):
                raise ValueError("order must be a permutation of range(B)")
            d.order = self._dev(torch.from_numpy(order))
        d.path = int(path)
        self.desc = d

    def _dev(self, t):
        t = t.to(self.device)
        self._keep.append(t)
        return t.data_ptr()

    @classmethod
    def uniform(cls, B, n, m, dtype=torch.float32, device="cuda", order=None, path=N.PATH_AUTO):
        return cls(B, dtype, device, n=n, m=m, order=order, path=path)

    @classmethod
    def packed_from(cls, nv, nrows, dtype=torch.float32, device="cuda", order=None,
                    path=N.PATH_AUTO):
        return cls(len(nv), dtype, device, nv=nv, nrows=nrows, order=order, path=path)

    # sizes -------------------------------------------------------------
    def sizes(self):
        return dict(M=self.total_nn, J=self.total_mn, a0=self.total_n, aref=self.total_m,
                    D=self.total_m, a=self.total_n, abar=self.total_n)

    def state_bytes(self) -> int:
        return N.state_bytes(self.desc)

    def mask_offset(self) -> int:
        """Byte offset of the active-set bytes inside the state buffer."""
        s = 4 if self.dtype == torch.float32 else 8
        return (s * (self.total_nn + self.total_n) // 2 + 255) // 256 * 256

    def active_sets(self, sol) -> np.ndarray:
        """Active set A* of every row (host copy, flat, off_m layout)."""
        o = self.mask_offset()
        return sol.state[o:o + self.total_m].cpu().numpy().astype(bool)

    def zones(self, sol) -> np.ndarray:
        """Round cone: each contact's zone (0, 1, 2) from the state written by
        cs_forward_ell (host copy, flat, off_m / 3 layout)."""
        o = self.mask_offset()
        return sol.state[o:o + self.total_m].cpu().numpy()[0::3].copy()

    def tape_bytes(self, K: int) -> int:
        return N.tape_bytes(self.desc, K)

    def check(self, name: str, t: Optional[torch.Tensor], numel: int, required=True):
        if t is None:
            if required:
                raise ValueError(f"{name} is required")
            return
        if t.device != self.device and not (t.device.type == self.device.type and
                                            self.device.index is None):
            raise ValueError(f"{name} is on {t.device}, batch is on {self.device}")
        if t.dtype != self.dtype:
            raise ValueError(f"{name} has dtype {t.dtype}, batch is {self.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != numel:
            raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


@dataclass
class Solution:
    a: torch.Tensor
    state: torch.Tensor       # uint8 device buffer (factor of H(A*) and A*)
    status: torch.Tensor      # int32 [B]
    iters: torch.Tensor       # int32 [B]


def forward(batch: Batch, M, J, a0, aref, D, *, max_iter=10, tol=1e-5, a_init=None,
            out: Optional[Solution] = None, method: str = "newton") -> Solution:
    """Forward solve; method "newton" (Newton steps) or "cg" (nonlinear
    conjugate gradients, SMALL-family batches only), both with the exact line
    search.  max_iter caps the steps of the chosen method."""
    if method not in ("newton", "cg"):
        raise ValueError(f"unknown method {method!r}")
    s = batch.sizes()
    for name, t in (("M", M), ("J", J), ("a0", a0), ("aref", aref), ("D", D)):
        batch.check(name, t, s[name])
    batch.check("a_init", a_init, s["a0"], required=False)
    if out is None:
        shape = a0.shape
        out = Solution(
            a=torch.empty(shape, dtype=batch.dtype, device=a0.device),
            state=torch.empty(max(batch.state_bytes(), 1), dtype=torch.uint8, device=a0.device),
            status=torch.empty(batch.B, dtype=torch.int32, device=a0.device),
            iters=torch.empty(batch.B, dtype=torch.int32, device=a0.device))
    batch.check("a_out", out.a, s["a"])
    if out.state.numel() < batch.state_bytes():
        raise ValueError("state buffer too small")
    p = N.CsSolverParams(int(max_iter), N.FORWARD_CG if method == "cg" else 0, float(tol))
    rc = N.forward(batch.desc, p, _vp(M), _vp(J), _vp(a0), _vp(aref), _vp(D), _vp(a_init),
                   _vp(out.a), _vp(out.state), out.state.numel(), _vp(out.status), _vp(out.iters),
                   _stream(a0.device))
    N.check(rc, "cs_forward")
    return out


def ift_vjp(batch: Batch, sol: Solution, M, J, a0, aref, D, abar,
            needs=(True, True, True, True, True), out=None):
    """Returns (a0bar, arefbar, Jbar, Dbar, Mbar); entries not needed are None."""
    s = batch.sizes()
    for name, t in (("M", M), ("J", J), ("a0", a0), ("aref", aref), ("D", D), ("abar", abar)):
        batch.check(name, t, s[name])
    like = {0: a0, 1: aref, 2: J, 3: D, 4: M}
    if out is None:
        out = tuple(torch.empty_like(like[k]) if needs[k] else None for k in range(5))
    for k, name in enumerate(("a0bar", "arefbar", "Jbar", "Dbar", "Mbar")):
        batch.check(name, out[k], like[k].numel(), required=False)
    rc = N.ift_vjp(batch.desc, _vp(sol.state), sol.state.numel(), _vp(M), _vp(J), _vp(a0),
                   _vp(aref), _vp(D), _vp(sol.a), _vp(abar), *(_vp(t) for t in out),
                   _stream(a0.device))
    N.check(rc, "cs_ift_vjp")
    return out


def forward_ell(batch: Batch, M, J, a0, aref, dn, dt, mu, *, max_iter=60, tol=1e-5,
                a_init=None, out: Optional[Solution] = None) -> Solution:
    """Round-cone forward solve (cs_forward_ell): rows (N, T1, T2) per contact,
    dn, dt, mu one value per contact (total_m / 3 each)."""
    s = batch.sizes()
    for name, t in (("M", M), ("J", J), ("a0", a0), ("aref", aref)):
        batch.check(name, t, s[name])
    ncon = s["aref"] // 3
    for name, t in (("dn", dn), ("dt", dt), ("mu", mu)):
        batch.check(name, t, ncon)
    batch.check("a_init", a_init, s["a0"], required=False)
    if out is None:
        out = Solution(
            a=torch.empty_like(a0),
            state=torch.empty(max(batch.state_bytes(), 1), dtype=torch.uint8, device=a0.device),
            status=torch.empty(batch.B, dtype=torch.int32, device=a0.device),
            iters=torch.empty(batch.B, dtype=torch.int32, device=a0.device))
    p = N.CsSolverParams(int(max_iter), 0, float(tol))
    rc = N.forward_ell(batch.desc, p, _vp(M), _vp(J), _vp(a0), _vp(aref), _vp(dn), _vp(dt), _vp(mu),
                       _vp(a_init), _vp(out.a), _vp(out.state), out.state.numel(), _vp(out.status),
                       _vp(out.iters), _stream(a0.device))
    N.check(rc, "cs_forward_ell")
    return out


def ift_vjp_ell(batch: Batch, sol: Solution, M, J, a0, aref, dn, dt, mu, abar, out=None):
    """Round-cone IFT VJP (cs_ift_vjp_ell).  Returns dict(a0, aref, J, dn, dt, mu, M)
    (`out`, when given, is filled and returned)."""
    s = batch.sizes()
    for name, t in (("M", M), ("J", J), ("a0", a0), ("aref", aref), ("abar", abar)):
        batch.check(name, t, s[name])
    if out is None:
        out = dict(a0=torch.empty_like(a0), aref=torch.empty_like(aref), J=torch.empty_like(J),
                   dn=torch.empty_like(dn), dt=torch.empty_like(dt), mu=torch.empty_like(mu),
                   M=torch.empty_like(M))
    rc = N.ift_vjp_ell(batch.desc, _vp(sol.state), sol.state.numel(), _vp(M), _vp(J), _vp(a0),
                       _vp(aref), _vp(dn), _vp(dt), _vp(mu), _vp(sol.a), _vp(abar), _vp(out["a0"]),
                       _vp(out["aref"]), _vp(out["J"]), _vp(out["dn"]), _vp(out["dt"]),
                       _vp(out["mu"]), _vp(out["M"]), _stream(a0.device))
    N.check(rc, "cs_ift_vjp_ell")
    return out


def forward_rows(batch: Batch, M, J, a0, aref, D, kind, floss, *, max_iter=60, tol=1e-5,
                 a_init=None, out: Optional[Solution] = None) -> Solution:
    """Mixed-row forward solve (cs_forward_rows): kind (uint8 per row: 0
    one-sided, 1 equality, 2 friction loss) and floss (the friction bound)
    at the row offsets."""
    s = batch.sizes()
    for name, t in (("M", M), ("J", J), ("a0", a0), ("aref", aref), ("D", D), ("floss", floss)):
        batch.check(name, t, s["D"] if name == "floss" else s[name])
    if kind.dtype != torch.uint8 or kind.numel() != s["D"] or not kind.is_contiguous():
        raise ValueError("kind must be a contiguous uint8 tensor with one byte per row")
    batch.check("a_init", a_init, s["a0"], required=False)
    if out is None:
        out = Solution(
            a=torch.empty_like(a0),
            state=torch.empty(max(batch.state_bytes(), 1), dtype=torch.uint8, device=a0.device),
            status=torch.empty(batch.B, dtype=torch.int32, device=a0.device),
            iters=torch.empty(batch.B, dtype=torch.int32, device=a0.device))
    p = N.CsSolverParams(int(max_iter), 0, float(tol))
    rc = N.forward_rows(batch.desc, p, _vp(M), _vp(J), _vp(a0), _vp(aref), _vp(D), _vp(kind),
                        _vp(floss), _vp(a_init), _vp(out.a), _vp(out.state), out.state.numel(),
                        _vp(out.status), _vp(out.iters), _stream(a0.device))
    N.check(rc, "cs_forward_rows")
    return out


def ift_vjp_rows(batch: Batch, sol: Solution, M, J, a0, aref, D, kind, floss, abar, out=None):
    """Mixed-row IFT VJP (cs_ift_vjp_rows).  Returns dict(a0, aref, J, D, floss, M)."""
    s = batch.sizes()
    for name, t in (("M", M), ("J", J), ("a0", a0), ("aref", aref), ("D", D), ("abar", abar)):
        batch.check(name, t, s[name])
    if out is None:
        out = dict(a0=torch.empty_like(a0), aref=torch.empty_like(aref), J=torch.empty_like(J),
                   D=torch.empty_like(D), floss=torch.empty_like(floss), M=torch.empty_like(M))
    rc = N.ift_vjp_rows(batch.desc, _vp(sol.state), sol.state.numel(), _vp(M), _vp(J), _vp(a0),
                        _vp(aref), _vp(D), _vp(kind), _vp(floss), _vp(sol.a), _vp(abar),
                        _vp(out["a0"]), _vp(out["aref"]), _vp(out["J"]), _vp(out["D"]),
                        _vp(out["floss"]), _vp(out["M"]), _stream(a0.device))
    N.check(rc, "cs_ift_vjp_rows")
    return out


def ift_jvp(batch: Batch, sol: Solution, M, J, D, k: int, da0=None, daref=None, out=None):
    """Directional derivatives of the solution for k tangent directions per
    instance (eq. 15): da0 [k * total_n] (instance i's k x n block at k off_n[i]),
    daref [k * total_m] (k x m at k off_m[i]), either None.  Returns da
    [k * total_n] in the same layout."""
    s = batch.sizes()
    for name, t in (("M", M), ("J", J), ("D", D)):
        batch.check(name, t, s[name])
    batch.check("da0", da0, k * s["a0"], required=False)
    batch.check("daref", daref, k * s["aref"], required=False)
    if out is None:
        out = torch.empty(max(k * s["a0"], 1), dtype=batch.dtype, device=M.device)
    rc = N.ift_jvp(batch.desc, _vp(sol.state), sol.state.numel(), _vp(M), _vp(J), _vp(D), int(k),
                   _vp(da0), _vp(daref), _vp(out), _stream(M.device))
    N.check(rc, "cs_ift_jvp")
    return out


def unrolled_record(batch: Batch, M, J, a0, aref, D, *, K=10, tol=1e-5, tape=None):
    """Run the K-step solve and record its trace.  Returns dict(a, status, iters, tape)."""
    s = batch.sizes()
    for name, t in (("M", M), ("J", J), ("a0", a0), ("aref", aref), ("D", D)):
        batch.check(name, t, s[name])
    nbytes = batch.tape_bytes(K)
    if tape is None:
        tape = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=a0.device)
    if tape.numel() < nbytes:
        raise ValueError("tape buffer too small")
    out = dict(a=torch.empty_like(a0),
               status=torch.empty(batch.B, dtype=torch.int32, device=a0.device),
               iters=torch.empty(batch.B, dtype=torch.int32, device=a0.device), tape=tape, K=K,
               tol=tol)
    p = N.CsSolverParams(int(K), N.UNROLLED_RECORD, float(tol))
    rc = N.unrolled_vjp(batch.desc, p, _vp(M), _vp(J), _vp(a0), _vp(aref), _vp(D), None,
                        _vp(out["a"]), None, None, None, None, None, _vp(tape), tape.numel(),
                        _vp(out["status"]), _vp(out["iters"]), _stream(a0.device))
    N.check(rc, "cs_unrolled_vjp(record)")
    return out


def unrolled_replay(batch: Batch, rec, M, J, a0, aref, D, abar,
                    needs=(True, True, True, True, True)):
    """Reverse sweep over a trace from unrolled_record.  Returns (a0bar, arefbar, Jbar, Dbar, Mbar)."""
    s = batch.sizes()
    for name, t in (("M", M), ("J", J), ("a0", a0), ("aref", aref), ("D", D), ("abar", abar)):
        batch.check(name, t, s[name])
    g = tuple(torch.empty_like(x) for x in (a0, aref, J, D, M))
    p = N.CsSolverParams(int(rec["K"]), N.UNROLLED_REPLAY, float(rec["tol"]))
    tape = rec["tape"]
    rc = N.unrolled_vjp(batch.desc, p, _vp(M), _vp(J), _vp(a0), _vp(aref), _vp(D), _vp(abar),
                        None, *(_vp(t) for t in g), _vp(tape), tape.numel(), _vp(rec["status"]),
                        _vp(rec["iters"]), _stream(a0.device))
    N.check(rc, "cs_unrolled_vjp(replay)")
    return tuple(x if need else None for x, need in zip(g, needs))


def unrolled_vjp(batch: Batch, M, J, a0, aref, D, abar, *, K=10, tol=1e-5, tape=None, out=None):
    """Unrolled-trace gradient of abar . a_K.  Returns dict(a, a0, aref, J, D, M, status, iters,
    tape_bytes); ``out``, a dict this function returned before for the same batch, is
    written in place."""
    s = batch.sizes()
    for name, t in (("M", M), ("J", J), ("a0", a0), ("aref", aref), ("D", D), ("abar", abar)):
        batch.check(name, t, s[name])
    nbytes = batch.tape_bytes(K)
    if tape is None:
        tape = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=a0.device)
    if tape.numel() < nbytes:
        raise ValueError("tape buffer too small")
    if out is None:
        out = dict(a=torch.empty_like(a0), a0=torch.empty_like(a0), aref=torch.empty_like(aref),
                   J=torch.empty_like(J), D=torch.empty_like(D), M=torch.empty_like(M),
                   status=torch.empty(batch.B, dtype=torch.int32, device=a0.device),
                   iters=torch.empty(batch.B, dtype=torch.int32, device=a0.device))
    p = N.CsSolverParams(int(K), 0, float(tol))
    rc = N.unrolled_vjp(batch.desc, p, _vp(M), _vp(J), _vp(a0), _vp(aref), _vp(D), _vp(abar),
                        _vp(out["a"]), _vp(out["a0"]), _vp(out["aref"]), _vp(out["J"]),
                        _vp(out["D"]), _vp(out["M"]), _vp(tape), tape.numel(), _vp(out["status"]),
                        _vp(out["iters"]), _stream(a0.device))
    N.check(rc, "cs_unrolled_vjp")
    out["tape_bytes"] = nbytes
    return out
