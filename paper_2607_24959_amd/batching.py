"""Uneven (packed) batches: tile classes, LPT order and graph capture.

A packed batch mixes instance shapes whose costs span orders of magnitude.
The planner sorts instances into tile classes (one kernel family and its
compile-time sizes per class), orders each class longest-processing-time
first by a cost model, and issues one cs_forward / cs_ift_vjp per class on
the same stream with ``order``/``count`` selecting the class's instances, so
the whole batch shares one set of buffers and one state.  The sequence can
be captured in a HIP graph and replayed, on one stream or with the classes
dealt to two streams that run concurrently inside the graph.

Class rules come from a table keyed by (dtype, padded n, row bucket); the
autotuner (autotune.py) fills it by timing the candidate families, and the
defaults below apply otherwise.
"""
from __future__ import annotations

import ctypes as C
import json
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
import torch

from . import _native as N
from . import solver

SMALL_NP = (3, 6, 9, 12)
SMALL_M = (16, 32, 64)
TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tile_table.json")


def n_bucket(n: int) -> int:
    for b in SMALL_NP:
        if n <= b:
            return b
    return (n + 15) // 16 * 16


def m_bucket(m: int) -> int:
    for b in SMALL_M:
        if m <= b:
            return b
    return (m + 63) // 64 * 64


def cost_model(n, m):
    """Relative cost of one solve: row passes (m n), Newton-matrix contraction on
    the active rows (~m/2, matrix cores) and the factorisation (n^3/3)."""
    n = np.asarray(n, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    return 4.0 * m * n + 0.25 * m * n * n + n ** 3 / 3.0 + 64.0


def default_family(dtype, n, m):
    s = 4 if dtype == torch.float32 else 8
    if m <= 64 and ((s == 4 and n <= 12) or (s == 8 and n <= 6)):
        return N.PATH_SMALL
    if s == 4 and n <= 31 and m <= 1024:
        return N.PATH_WAVE
    if n <= 128 and m <= 2048:
        return N.PATH_CHUNK
    return N.PATH_TEAM


def load_table(path: str = TABLE_PATH) -> Dict[str, int]:
    if os.path.exists(path):
        with open(path) as f:
            return {k: int(v) for k, v in json.load(f).get("families", {}).items()}
    return {}


def table_key(dtype, nb, mb):
    return f"{'f32' if dtype == torch.float32 else 'f64'}:n{nb}:m{mb}"


@dataclass
class TileClass:
    path: int
    idx: np.ndarray          # instance indices, LPT order
    nmax: int
    mmax: int
    order_dev: Optional[torch.Tensor] = None
    desc: Optional[N.CsBatch] = None


class Plan:
    """Execution plan of one packed batch (shapes fixed; values may change)."""

    def __init__(self, batch: solver.Batch, table: Optional[Dict[str, int]] = None,
                 lpt: bool = True, families: Optional[Dict[str, int]] = None):
        self.batch = batch
        table = load_table() if table is None else table
        if families:
            table = dict(table, **families)
        nv, nr = batch.nv_host, batch.nrows_host
        groups: Dict[tuple, List[int]] = {}
        for i in range(batch.B):
            n, m = int(nv[i]), int(nr[i])
            key = table_key(batch.dtype, n_bucket(n), m_bucket(m))
            fam = table.get(key, default_family(batch.dtype, n, m))
            if fam == N.PATH_SMALL:
                gk = (fam, n_bucket(n), m_bucket(m))
            elif fam == N.PATH_CHUNK:
                gk = (fam, 0 if n <= 32 else 1, 0)   # one launch per workgroup size
            elif fam == N.PATH_WAVE:
                gk = (fam, 0 if n <= 15 else 1, 0)   # one launch per padded width
            else:
                gk = (fam, 0, 0)
            groups.setdefault(gk, []).append(i)
        self.classes: List[TileClass] = []
        for gk in sorted(groups, key=lambda g: -cost_model(nv[groups[g]], nr[groups[g]]).sum()):
            idx = np.asarray(groups[gk], dtype=np.int64)
            if lpt:
                idx = idx[np.argsort(-cost_model(nv[idx], nr[idx]), kind="stable")]
            tc = TileClass(path=gk[0], idx=idx.astype(np.int32), nmax=int(nv[idx].max()),
                           mmax=int(nr[idx].max()))
            tc.order_dev = torch.from_numpy(tc.idx).to(batch.device)
            d = N.CsBatch()
            C.memmove(C.byref(d), C.byref(batch.desc), C.sizeof(N.CsBatch))
            d.order = tc.order_dev.data_ptr()
            d.count = len(tc.idx)
            d.path = tc.path
            if d.nv:                    # packed: class maxima
                d.nv_max, d.nrows_max = tc.nmax, tc.mmax
            tc.desc = d
            self.classes.append(tc)
        self.graph = None

    def summary(self):
        return [dict(path=c.path, count=len(c.idx), nmax=c.nmax, mmax=c.mmax) for c in self.classes]

    # ------------------------------------------------------------------ calls
    def forward(self, M, J, a0, aref, D, *, max_iter, tol, out: Optional[solver.Solution] = None):
        b = self.batch
        if out is None:
            out = solver.Solution(
                a=torch.empty_like(a0),
                state=torch.empty(max(b.state_bytes(), 1), dtype=torch.uint8, device=a0.device),
                status=torch.empty(b.B, dtype=torch.int32, device=a0.device),
                iters=torch.empty(b.B, dtype=torch.int32, device=a0.device))
        s = b.sizes()
        for name, t in (("M", M), ("J", J), ("a0", a0), ("aref", aref), ("D", D)):
            b.check(name, t, s[name])
        p = N.CsSolverParams(int(max_iter), 0, float(tol))
        vp = solver._vp
        st = solver._stream(a0.device)
        for c in self.classes:
            rc = N.forward(c.desc, p, vp(M), vp(J), vp(a0), vp(aref), vp(D), None, vp(out.a),
                           vp(out.state), out.state.numel(), vp(out.status), vp(out.iters), st)
            N.check(rc, f"cs_forward(class path={c.path})")
        return out

    def ift_vjp(self, sol, M, J, a0, aref, D, abar, out=None):
        b = self.batch
        if out is None:
            out = tuple(torch.empty_like(x) for x in (a0, aref, J, D, M))
        vp = solver._vp
        st = solver._stream(a0.device)
        for c in self.classes:
            rc = N.ift_vjp(c.desc, vp(sol.state), sol.state.numel(), vp(M), vp(J), vp(a0),
                           vp(aref), vp(D), vp(sol.a), vp(abar), *(vp(t) for t in out), st)
            N.check(rc, f"cs_ift_vjp(class path={c.path})")
        return out

    # ------------------------------------------------------------------ lanes
    def lane_split(self, lanes: int) -> List[List[int]]:
        """Classes dealt to `lanes` streams longest first, each to the lane with
        the least estimated work (cost model summed over the class)."""
        nv, nr = self.batch.nv_host, self.batch.nrows_host
        cost = [float(cost_model(nv[c.idx], nr[c.idx]).sum()) for c in self.classes]
        out: List[List[int]] = [[] for _ in range(lanes)]
        load = [0.0] * lanes
        for ci in sorted(range(len(self.classes)), key=lambda i: -cost[i]):
            k = int(np.argmin(load))
            out[k].append(ci)
            load[k] += cost[ci]
        return out

    def _issue(self, t, sol, grads, max_iter, tol, classes, stream):
        """Forward then VJP of each listed class on `stream` (classes touch
        disjoint instances, so lanes need no ordering between them)."""
        vp = solver._vp
        p = N.CsSolverParams(int(max_iter), 0, float(tol))
        st = C.c_void_p(stream.cuda_stream)
        for ci in classes:
            c = self.classes[ci]
            rc = N.forward(c.desc, p, vp(t["M"]), vp(t["J"]), vp(t["a0"]), vp(t["aref"]), vp(t["D"]),
                           None, vp(sol.a), vp(sol.state), sol.state.numel(), vp(sol.status),
                           vp(sol.iters), st)
            N.check(rc, f"cs_forward(class path={c.path})")
            if grads is not None:
                rc = N.ift_vjp(c.desc, vp(sol.state), sol.state.numel(), vp(t["M"]), vp(t["J"]),
                               vp(t["a0"]), vp(t["aref"]), vp(t["D"]), vp(sol.a), vp(t["abar"]),
                               *(vp(x) for x in grads), st)
                N.check(rc, f"cs_ift_vjp(class path={c.path})")

    # ------------------------------------------------------------------ graphs
    def capture(self, tensors, *, max_iter, tol, with_vjp=True, lanes=1):
        """Capture forward (+ IFT VJP) of every class into one HIP graph.  With
        lanes = 2 the classes are dealt to two streams (lane_split) that run
        concurrently inside the graph, so small classes fill the compute units
        the longest class leaves idle; the streams stay alive with the graph."""
        t = tensors
        sol = self.forward(t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=max_iter, tol=tol)
        grads = self.ift_vjp(sol, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"]) if with_vjp else None
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        streams = [torch.cuda.Stream() for _ in range(lanes)]    # default priority
        split = self.lane_split(lanes)
        cap = streams[0]
        cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cap):
            with torch.cuda.graph(g, stream=cap):
                for st in streams[1:]:
                    st.wait_stream(cap)
                for k, st in enumerate(streams):
                    self._issue(t, sol, grads, max_iter, tol, split[k], st)
                for st in streams[1:]:
                    cap.wait_stream(st)
        torch.cuda.current_stream().wait_stream(cap)
        torch.cuda.synchronize()
        self.graph = g
        self.graph_streams = streams
        self.lanes = lanes
        return sol, grads
