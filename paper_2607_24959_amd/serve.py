"""Continuous-batching engine for MPC-window requests.

A request is one W-step window of the semi-implicit rollout that the
paper's trajectory optimisation and short-horizon residual MPC run (Sec.
IV-A, Sec. V): W forward contact solves with v_{t+1} = v_t + h a_t, then W
IFT VJPs in reverse for the gradient of ||v_W - v_goal||^2 w.r.t. the
actuation tau_t of every step.

The engine keeps a fixed table of S slots in device memory, each with room
for the largest request shape (n_cap, m_cap); S follows from an HBM budget.
Every tick it
  1. admits queued requests into free slots (cs_serve_admit),
  2. prepares every occupied slot's step (cs_serve_pre): the forward inputs
     a0 = M^{-1} tau_t, aref = -b J v_t - k pen, or, in the backward phase,
     the solution, factor and active set of step t restored from the
     per-step archive, so factorisations stay on the device and are reused,
  3. runs one cs_ift_vjp per kernel class over the slots in a backward phase
     and one cs_forward per class over the slots in a forward phase,
  4. consumes the outputs (cs_serve_post): archive, v += h a, or the
     gradient recursion, and advances every slot's phase on the host.
Requests at different phases share launches; admission needs only a free
slot, so new work overlaps with work already on the device.  The host side
of a tick is its bookkeeping and one native call (cs_serve_tick) that
uploads the tick's index lists from pinned memory and enqueues steps 1-4;
the host waits for the previous tick to start on the device, so it runs
one tick ahead.  An instance's arithmetic
does not depend on its slot or on the other slots (kernel classes have fixed
compile-time sizes), so a request's result is the same alone and in any mix.
"""
from __future__ import annotations

import ctypes as C
import gc
import time
from collections import deque
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np
import torch

from . import _native as N
from . import batching, solver, synth


@dataclass
class Request:
    rid: int
    pool_index: int
    n: int
    m: int
    arrival: float = 0.0          # seconds on the engine clock
    admitted: float = -1.0
    done: float = -1.0
    done_tick: int = -1


def slot_bytes(n_cap, m_cap, window, s=4):
    """Device bytes one slot holds (payload, request state, work arrays, archive)."""
    ne = n_cap * (n_cap + 1) // 2
    vals = (2 * n_cap * n_cap + m_cap * n_cap + 2 * m_cap      # M, M^-1, J, D, pen
            + 7 * n_cap + 2 * window * n_cap                   # v, goal, vbar, a0, abar, a, a0bar; tau, taubar
            + 2 * m_cap + ne                                   # aref, arefbar; factor
            + window * (2 * n_cap + m_cap + ne))               # archived a, a0, aref, factor
    return vals * s + (window + 1) * m_cap + 128               # active sets; sizes, offsets, status, lists


def _dt(dtype):
    return N.CS_F32 if dtype == torch.float32 else N.CS_F64


class RequestPool:
    """Device-resident request payloads (seeded synthetic), in the slot layout.

    ``Mp``/``Jp`` keep padded copies ([P, n_cap, n_cap] with an identity block,
    [P, m_cap, n_cap]) for references outside the engine."""

    def __init__(self, count, n_choices, nc_max, window, seed, n_cap, m_cap, dtype, device):
        rng = np.random.Generator(np.random.PCG64(seed))
        self.n = rng.choice(np.asarray(n_choices), size=count).astype(np.int32)
        self.nc = rng.integers(0, nc_max + 1, size=count).astype(np.int32)
        self.m = (synth.ROWS_PER_CONTACT * self.nc).astype(np.int32)
        if self.n.max() > n_cap or self.m.max() > m_cap:
            raise ValueError("pool shapes exceed the slot capacity")
        P = count
        Mt = np.zeros((P, n_cap * n_cap))
        Jt = np.zeros((P, m_cap * n_cap))
        Mp = np.tile(np.eye(n_cap), (P, 1, 1)); Jp = np.zeros((P, m_cap, n_cap))
        D = np.zeros((P, m_cap)); pen = np.zeros((P, m_cap))
        v0 = np.zeros((P, n_cap)); goal = np.zeros((P, n_cap)); tau = np.zeros((P, window, n_cap))
        for i in range(P):
            n, nc, m = int(self.n[i]), int(self.nc[i]), int(self.m[i])
            d = synth.instance(seed, i, n, nc)
            r2 = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, i, 1])))
            Mt[i, :n * n] = d["M"].ravel()
            Jt[i, :m * n] = d["J"].ravel()
            Mp[i, :n, :n] = d["M"]
            Jp[i, :m, :n] = d["J"]
            D[i, :m] = d["D"]
            pen[i, :m] = np.repeat(d["pen"], synth.ROWS_PER_CONTACT)
            v0[i, :n] = r2.standard_normal(n)
            goal[i, :n] = r2.standard_normal(n)
            tau[i, :, :n] = r2.standard_normal((window, n))
        self.n_cap, self.m_cap, self.W, self.dtype = n_cap, m_cap, window, dtype
        t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(device, dtype)
        self.Mt, self.Jt, self.Mp, self.Jp = t(Mt), t(Jt), t(Mp), t(Jp)
        Minv_p = torch.linalg.inv(self.Mp)          # block diagonal: inv(M) and the identity
        self.Minv = torch.zeros_like(self.Mt)
        for i in range(P):
            n = int(self.n[i])
            self.Minv[i, :n * n] = Minv_p[i, :n, :n].reshape(-1)
        self.D, self.pen = t(D), t(pen)
        self.v0, self.goal, self.tau = t(v0), t(goal), t(tau)
        self.nv = torch.from_numpy(self.n).to(device)
        self.nrows = torch.from_numpy(self.m).to(device)
        tb = N.CsServeTable()
        tb.dtype, tb.slots, tb.window = _dt(dtype), P, window
        tb.n_cap, tb.m_cap = n_cap, m_cap
        vp = lambda x: x.data_ptr()
        tb.M, tb.Minv, tb.J, tb.D, tb.pen = vp(self.Mt), vp(self.Minv), vp(self.Jt), vp(self.D), vp(self.pen)
        tb.v, tb.goal, tb.tau = vp(self.v0), vp(self.goal), vp(self.tau)
        tb.nv, tb.nrows = vp(self.nv), vp(self.nrows)
        self.table = tb


class Engine:
    def __init__(self, *, n_cap=18, m_cap=256, window=6, h=0.002, slots=None,
                 budget_bytes=None, max_iter=10, tol=1e-5, dtype=torch.float32, device="cuda"):
        self.n_cap, self.m_cap, self.W, self.h = n_cap, m_cap, window, h
        self.max_iter, self.tol, self.dtype = max_iter, tol, dtype
        self.device = dev = torch.device(device)
        s = 4 if dtype == torch.float32 else 8
        self.bytes_per_slot = slot_bytes(n_cap, m_cap, window, s)
        if slots is None:
            if budget_bytes is None:
                raise ValueError("give slots or budget_bytes")
            slots = int(budget_bytes // self.bytes_per_slot)
        if slots < 1:
            raise ValueError("the HBM budget does not hold one request slot")
        if n_cap > 64:
            raise ValueError("n_cap is limited to 64")
        self.S = S = int(slots)
        dt = dtype
        z = lambda *shape: torch.zeros(shape, dtype=dt, device=dev)
        ne = n_cap * (n_cap + 1) // 2
        self.M, self.Minv = z(S, n_cap * n_cap), z(S, n_cap * n_cap)
        self.J, self.D, self.pen = z(S, m_cap * n_cap), z(S, m_cap), z(S, m_cap)
        self.v, self.goal, self.vbar = z(S, n_cap), z(S, n_cap), z(S, n_cap)
        self.tau, self.taubar = z(S, window, n_cap), z(S, window, n_cap)
        self.a0, self.abar, self.a0bar = z(S, n_cap), z(S, n_cap), z(S, n_cap)
        self.aref, self.arefbar = z(S, m_cap), z(S, m_cap)
        self.arch_a, self.arch_a0 = z(window, S, n_cap), z(window, S, n_cap)
        self.arch_aref, self.arch_fac = z(window, S, m_cap), z(window, S, ne)
        self.arch_mask = torch.zeros((window, S, m_cap), dtype=torch.uint8, device=dev)
        # the slot table as a packed batch with capacity offsets and live sizes
        self.nv_host = np.ones(S, dtype=np.int32)
        self.nr_host = np.zeros(S, dtype=np.int32)
        self.batch = solver.Batch.packed_from(np.full(S, n_cap), np.full(S, m_cap), dt, device=dev)
        self.nv_dev = torch.ones(S, dtype=torch.int32, device=dev)
        self.nr_dev = torch.zeros(S, dtype=torch.int32, device=dev)
        self.batch.desc.nv = self.nv_dev.data_ptr()
        self.batch.desc.nrows = self.nr_dev.data_ptr()
        self.sol = solver.Solution(
            a=z(S, n_cap), state=torch.zeros(self.batch.state_bytes(), dtype=torch.uint8, device=dev),
            status=torch.zeros(S, dtype=torch.int32, device=dev),
            iters=torch.zeros(S, dtype=torch.int32, device=dev))
        tb = N.CsServeTable()
        tb.dtype, tb.slots, tb.window, tb.n_cap, tb.m_cap = _dt(dt), S, window, n_cap, m_cap
        tb.h, tb.b_damp, tb.k_spring = h, synth.B_DAMP, synth.K_SPRING
        vp = lambda x: x.data_ptr()
        tb.M, tb.Minv, tb.J, tb.D, tb.pen = vp(self.M), vp(self.Minv), vp(self.J), vp(self.D), vp(self.pen)
        tb.v, tb.goal, tb.tau = vp(self.v), vp(self.goal), vp(self.tau)
        tb.nv, tb.nrows = vp(self.nv_dev), vp(self.nr_dev)
        tb.vbar, tb.taubar = vp(self.vbar), vp(self.taubar)
        tb.a0, tb.abar, tb.a, tb.a0bar = vp(self.a0), vp(self.abar), vp(self.sol.a), vp(self.a0bar)
        tb.aref, tb.arefbar = vp(self.aref), vp(self.arefbar)
        tb.state, tb.mask_offset = vp(self.sol.state), self.batch.mask_offset()
        tb.arch_a, tb.arch_a0, tb.arch_aref = vp(self.arch_a), vp(self.arch_a0), vp(self.arch_aref)
        tb.arch_fac, tb.arch_mask = vp(self.arch_fac), vp(self.arch_mask)
        self.table = tb
        # per-tick index lists: admit pairs, step entries, launch orders
        self.cap_list = 6 * S + 16
        self.list_dev = torch.zeros(self.cap_list, dtype=torch.int32, device=dev)
        pin = dev.type == "cuda"
        self.list_pin = [torch.zeros(self.cap_list, dtype=torch.int32, pin_memory=pin)
                         for _ in range(2)]
        self.list_evt = [None, None]
        self.list_ev_obj = [torch.cuda.Event(), torch.cuda.Event()] if pin else [None, None]
        self.ring = 0
        # the kernel launches of one tick touch disjoint slots, so they run
        # concurrently on two lanes -- the caller's stream and one side
        # stream (default priority) -- between the tick's pre and post kernels
        # on the caller's stream.  One side stream: every fork or join costs
        # the host a stream-wait call of ~12 us, and two lanes already hold
        # the widest forward apart from the rest.
        # The two lanes are taken from torch's stream pool one after the
        # other: run_stream runs on the first and the side lane is the
        # second.  (A serving run on the caller's stream, with a side stream
        # taken whenever an engine was made, was ~1.8x slower per tick in
        # some runs of a process that had made other streams before: the
        # two lanes then seemed to share one hardware queue.)
        self.lanes = [torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)] if pin else []
        self.side = self.lanes[1:]
        self.ev_pre = torch.cuda.Event() if pin else None
        self.ev_side = [torch.cuda.Event() for _ in self.side]
        self.params = N.CsSolverParams(int(max_iter), 0, float(tol))
        # raw pointers of the solver outputs the table does not hold, made once
        cp = lambda t: C.c_void_p(t.data_ptr())
        self._p = dict(status=cp(self.sol.status), iters=cp(self.sol.iters))
        # host bookkeeping
        self.phase = np.full(S, -1, dtype=np.int64)   # -1 free; 0..W-1 forward; W..2W-1 backward
        self.cls = np.zeros(S, dtype=np.int64)        # kernel class of the slot's request
        self.req: List[Optional[Request]] = [None] * S
        self.free = deque(range(S))
        self.queue: deque = deque()
        self.finished: List[Request] = []
        self.pool: Optional[RequestPool] = None
        self.results: Dict[int, torch.Tensor] = {}
        self.keep_results = False
        self.max_active = 0
        self.ticks = 0
        self._stream = None
        self.classes = self._class_table()
        # one batch descriptor per class (the library reads it during the
        # call, so it is reused; each launch sets its order list and count)
        self.class_desc = []
        for path, nmax, mmax in self.classes:
            d = N.CsBatch()
            C.memmove(C.byref(d), C.byref(self.batch.desc), C.sizeof(N.CsBatch))
            d.path, d.nv_max, d.nrows_max = path, nmax, mmax
            self.class_desc.append(d)
        self.class_arr = (N.CsBatch * len(self.class_desc))(*self.class_desc)
        # a tick's launches, rows of (kind, class, lane, count, order); at most
        # one forward and one VJP launch per class
        self.launch_rows = np.zeros((2 * len(self.classes), 5), dtype=np.int32)
        self._launch_ptr = self.launch_rows.ctypes.data
        self.list_np = [b.numpy() for b in self.list_pin]
        self._list_host = [b.data_ptr() for b in self.list_pin]
        self._list_dev = self.list_dev.data_ptr()
        self._ev = None
        if pin:
            # one record each makes the events, so their HIP handles exist
            s0 = torch.cuda.current_stream(dev)
            for ev in self.list_ev_obj + [self.ev_pre] + self.ev_side:
                ev.record(s0)
            self._ev = ([e.cuda_event for e in self.list_ev_obj], self.ev_pre.cuda_event,
                        self.ev_side[0].cuda_event)

    # ------------------------------------------------------------ setup
    def _class_table(self):
        """Kernel classes with compile-time sizes fixed per class: small-family
        classes by padded n with the 64-row layout, chunked classes by
        workgroup size, each launched with the class's maximum sizes."""
        out = []
        s = 4 if self.dtype == torch.float32 else 8
        for npad in batching.SMALL_NP:
            if npad <= self.n_cap and ((s == 4 and npad <= 12) or (s == 8 and npad <= 6)):
                out.append((N.PATH_SMALL, npad, min(64, self.m_cap)))
        if s == 4:   # the one-wave family: n <= 31, up to 1024 rows
            wm = min(1024, self.m_cap)
            out.append((N.PATH_WAVE, min(15, self.n_cap), wm))
            if self.n_cap > 15:
                out.append((N.PATH_WAVE, min(31, self.n_cap), wm))
        if s == 8 or self.m_cap > 1024 or self.n_cap > 31:
            out.append((N.PATH_CHUNK, min(32, self.n_cap), self.m_cap))
        if self.n_cap > 32:
            out.append((N.PATH_CHUNK, self.n_cap, self.m_cap))
        return out

    def class_of(self, n, m):
        fam = batching.default_family(self.dtype, n, m)
        for c, (path, nmax, mmax) in enumerate(self.classes):
            if path == fam and n <= nmax and m <= mmax:
                return c
        raise ValueError(f"no kernel class for n={n}, m={m}")

    def attach_pool(self, pool: RequestPool):
        if (pool.n_cap, pool.m_cap, pool.W, pool.dtype) != (self.n_cap, self.m_cap, self.W, self.dtype):
            raise ValueError("pool capacity, window or dtype differs from the engine's")
        self.pool = pool

    def submit(self, req: Request):
        if req.n > self.n_cap or req.m > self.m_cap:
            raise ValueError("request larger than a slot")
        self.queue.append(req)

    def active(self):
        return self.S - len(self.free)

    # ------------------------------------------------------------ a tick
    def tick(self, now):
        """Admit, then one batched backward and one batched forward step for
        every occupied slot.  Returns (solves issued, slots finished)."""
        W = self.W
        adm_s, adm_p = [], []
        while self.queue and self.free and self.queue[0].arrival <= now:
            r = self.queue.popleft()
            s = self.free.popleft()
            r.admitted = now
            self.req[s] = r
            self.phase[s] = 0
            self.nv_host[s], self.nr_host[s] = r.n, r.m
            self.cls[s] = self.class_of(r.n, r.m)
            adm_s.append(s)
            adm_p.append(r.pool_index)
        occ = np.flatnonzero(self.phase >= 0)
        self.max_active = max(self.max_active, len(occ))
        if len(occ) == 0:
            return 0, np.zeros(0, dtype=np.int64)
        ph = self.phase[occ]
        bwd_mask = ph >= W
        # list layout: [admit pairs | entries | orders of each launch]
        parts = [np.stack([np.asarray(adm_s, np.int64), np.asarray(adm_p, np.int64)], 1).ravel(),
                 np.stack([occ, ph], 1).ravel()]
        launches = []
        pos = 2 * len(adm_s) + 2 * len(occ)
        for kind, sel in (("vjp", occ[bwd_mask]), ("fwd", occ[~bwd_mask])):
            if len(sel) == 0:
                continue
            cs = self.cls[sel]
            for c in np.unique(cs):
                idx = sel[cs == c]
                parts.append(idx)
                launches.append((kind, int(c), pos, len(idx)))
                pos += len(idx)
        flat = np.concatenate(parts).astype(np.int32)
        # wait until the previous tick has started on the device (its list
        # upload, the first thing it enqueued, is done): the host then stays
        # one tick ahead, enough to keep the device busy while preparing a
        # tick takes less than running one, and a new request queues behind
        # one tick at most.  The upload of two ticks ago, which filled this
        # ring buffer, completed before it.
        ring = self.ring
        if self.list_evt[ring ^ 1] is not None:
            self.list_evt[ring ^ 1].synchronize()
        self.list_np[ring][:len(flat)] = flat
        self.list_evt[ring] = self.list_ev_obj[ring]
        self.ring ^= 1
        # the stream run_stream fixed for its run (looking it up costs the
        # host ~12 us a call), else the current one
        stream = self._stream if self._stream is not None else torch.cuda.current_stream(self.device)
        two = len(launches) > 1 and bool(self.side)
        deal_lanes(launches, self.classes, two, self.launch_rows)
        evl, evf, evj = self._ev
        rc = N.serve_tick(self.table, self.pool.table if adm_s else None, self.class_arr,
                          len(self.classes), self.params, self.sol.state.numel(),
                          self._p["status"], self._p["iters"], self._list_host[ring],
                          self._list_dev, len(flat), len(adm_s), len(occ), self._launch_ptr,
                          len(launches), stream.cuda_stream,
                          self.side[0].cuda_stream if two else None, evl[ring], evf, evj)
        N.check(rc, "cs_serve_tick")
        self.phase[occ] += 1
        done = occ[self.phase[occ] == 2 * W]
        self.ticks += 1
        for s in done:
            r = self.req[s]
            r.done_tick = self.ticks
            if self.keep_results:
                # on the tick's stream: after this tick's last kernel, before
                # the next tick's admission can reuse the slot
                n = r.n
                with torch.cuda.stream(stream):
                    self.results[r.rid] = torch.cat([self.v[s, :n], self.taubar[s, :, :n].reshape(-1)]).clone()
            self.req[s] = None
            self.phase[s] = -1
            self.free.append(s)
            self.finished.append(r)
        return len(occ), done


def deal_lanes(launches, classes, two, rows):
    """Order a tick's launches and pick their lanes.

    ``launches`` holds (kind, class, order offset, count) tuples with kind
    "fwd" or "vjp"; ``classes`` the engine's (family, n_max, m_max) table.
    Longest launches go first, each to the less loaded of the two lanes
    (lane 0 on ties, and always when ``two`` is false) by a latency estimate:
    a class launch of a few instances takes about one instance's solve, which
    grows with the class's n_max for a forward.  Fills ``rows[:len]`` with
    (kind 0 forward / 1 VJP, class, lane, count, order) and sorts
    ``launches`` in place."""
    est = lambda L: ((2.0 * classes[L[1]][1] + 40.0) if L[0] == "fwd" else 20.0)
    launches.sort(key=est, reverse=True)
    load = [0.0, 0.0]
    for i, L in enumerate(launches):
        k = 1 if two and load[1] < load[0] else 0
        load[k] += est(L)
        rows[i] = (0 if L[0] == "fwd" else 1, L[1], k, L[3], L[2])
    return rows[:len(launches)]


def run_stream(engine: Engine, rate, n_requests, warmup=0, seed=0):
    """Serve a Poisson stream of ``rate`` requests/s on the wall clock.

    The host issues each tick once the previous one has started on the GPU
    (one tick ahead of the device); every tick records a timing event, and a
    request completes when the event of its last tick completes on the GPU.
    Latency is measured from arrival to that completion on one clock.
    Returns percentiles over the requests after the warm-up ones, and
    throughput in requests and solves per second."""
    rng = np.random.default_rng(seed)
    total = n_requests + warmup
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=total))
    P = engine.pool
    pick = rng.integers(0, len(P.n), size=total)
    reqs = [Request(rid=i, pool_index=int(pick[i]), n=int(P.n[pick[i]]), m=int(P.m[pick[i]]),
                    arrival=float(arrivals[i])) for i in range(total)]
    pending = deque(reqs)
    engine.finished.clear()
    stream = engine.lanes[0] if engine.lanes else torch.cuda.current_stream(engine.device)
    engine._stream = stream
    # the loop allocates an event per tick; a cyclic-GC pass over the
    # growing heap would stall the host for milliseconds mid-stream
    gc_was_enabled = gc.isenabled()
    gc.collect()
    gc.disable()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    t0 = time.perf_counter()
    # one timing event per tick from a recycled pool: an event is read once
    # it is LAG ticks old (long complete by then) and reused, so a run makes
    # a bounded number of events instead of one per tick
    LAG = 64
    t_end = [0.0]                       # seconds since start, per tick
    in_flight: deque = deque()          # (tick number, event)
    spare: deque = deque()
    solves = 0
    t_first = engine.ticks

    def read_oldest():
        i, e = in_flight.popleft()
        t_end[i] = start.elapsed_time(e) / 1e3
        spare.append(e)

    while len(engine.finished) < total:
        now = time.perf_counter() - t0
        while pending and pending[0].arrival <= now:
            engine.submit(pending.popleft())
        if engine.active() == 0 and not engine.queue:
            continue                                    # idle: wait for the next arrival
        before = engine.ticks
        n_work, _ = engine.tick(now)
        if engine.ticks != before:
            ev = spare.popleft() if spare else torch.cuda.Event(enable_timing=True)
            ev.record(stream)
            t_end.append(0.0)
            in_flight.append((len(t_end) - 1, ev))
            if len(in_flight) > LAG:
                in_flight[0][1].synchronize()
                read_oldest()
            solves += n_work
    torch.cuda.synchronize()
    while in_flight:
        read_oldest()
    engine._stream = None
    if gc_was_enabled:
        gc.enable()
    for r in engine.finished:
        r.done = t_end[r.done_tick - t_first]
    fin = sorted(engine.finished, key=lambda r: r.rid)[warmup:]
    lat = np.array([r.done - r.arrival for r in fin])
    span = max(r.done for r in fin) - min(r.arrival for r in fin)
    return dict(rate=rate, requests=len(fin), p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3), requests_per_s=len(fin) / span,
                solves_per_s=solves / t_end[-1], ticks=len(t_end) - 1, slots=engine.S,
                max_active=engine.max_active)
