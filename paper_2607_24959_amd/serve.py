"""Continuous-batching engine for MPC-window requests.

A request is one W-step window of the semi-implicit rollout (the model of
rollout.py): W forward contact solves with v_{t+1} = v_t + h a_t, then W IFT
VJPs in reverse for the gradient of ||v_W - v_goal||^2 w.r.t. the actuation
tau of every step.

The engine keeps a fixed table of S slots in device memory, each with room
for the largest request shape (n_cap, m_cap); S follows from an HBM budget.
Every tick it
  1. admits queued requests into free slots (device-to-device copies),
  2. runs one batched cs_ift_vjp per kernel family over all slots in a
     backward phase, after restoring each slot's saved factor of H(A*) for
     its step from the per-step archive (factorisations stay on device),
  3. runs one batched cs_forward per kernel family over all slots in a
     forward phase and archives each slot's solution, factor and active set,
  4. advances every slot's phase; finished requests free their slot.
Requests at different phases share launches, and newly admitted work
overlaps with work already on the device.  An instance's arithmetic does not
depend on its slot or on the other slots, so a request's result is the same
alone and in any mix.

Slot layout: matrices are kept twice, tightly packed at the slot's offset
for the kernels (M: first n^2 of n_cap^2 elements, J: first m n of
m_cap n_cap) and padded ([n_cap, n_cap] with an identity block, [m_cap,
n_cap] with zeros) for the dense torch glue; vectors are padded at the end,
which is both layouts at once.
"""
from __future__ import annotations

import ctypes as C
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


def slot_bytes(n_cap, m_cap, window, s=4):
    """Device bytes one slot holds (inputs, per-step archive, work and outputs)."""
    ne = n_cap * (n_cap + 1) // 2
    vals = (3 * n_cap * n_cap + 2 * m_cap * n_cap + 2 * m_cap      # M tight/padded/inverse, J x2, D, pen
            + 6 * n_cap + 2 * window * n_cap                      # v, goal, vbar, a0, abar, mask, tau, tau-bar
            + window * (2 * n_cap + m_cap + ne)                   # archived a, a0, aref, factor
            + 2 * n_cap + 2 * m_cap + ne)                         # work a, grads, aref, factor
    return vals * s + (window + 1) * m_cap                        # archived and work active sets


class RequestPool:
    """Device-resident request payloads (seeded synthetic) in both slot layouts."""

    def __init__(self, count, n_choices, nc_max, window, seed, n_cap, m_cap, dtype, device):
        rng = np.random.Generator(np.random.PCG64(seed))
        self.n = rng.choice(np.asarray(n_choices), size=count).astype(np.int32)
        self.nc = rng.integers(0, nc_max + 1, size=count).astype(np.int32)
        self.m = (synth.ROWS_PER_CONTACT * self.nc).astype(np.int32)
        P = count
        Mt = np.zeros((P, n_cap * n_cap)); Jt = np.zeros((P, m_cap * n_cap))
        Mp = np.tile(np.eye(n_cap), (P, 1, 1)); Jp = np.zeros((P, m_cap, n_cap))
        D = np.zeros((P, m_cap)); pen = np.zeros((P, m_cap)); nmask = np.zeros((P, n_cap))
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
            nmask[i, :n] = 1.0
            v0[i, :n] = r2.standard_normal(n)
            goal[i, :n] = r2.standard_normal(n)
            tau[i, :, :n] = r2.standard_normal((window, n))
        t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(device, dtype)
        self.Mt, self.Jt, self.Mp, self.Jp = t(Mt), t(Jt), t(Mp), t(Jp)
        self.Minv = torch.linalg.inv(self.Mp)
        self.D, self.pen, self.nmask = t(D), t(pen), t(nmask)
        self.v0, self.goal, self.tau = t(v0), t(goal), t(tau)


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
        self.S = S = int(slots)
        dt = dtype
        z = lambda *shape: torch.zeros(shape, dtype=dt, device=dev)
        ne = n_cap * (n_cap + 1) // 2
        # kernel layout (tight at the slot offset) and glue layout (padded)
        self.Mt, self.Jt = z(S, n_cap * n_cap), z(S, m_cap * n_cap)
        self.Minv, self.Jp = z(S, n_cap, n_cap), z(S, m_cap, n_cap)
        self.D, self.pen, self.nmask = z(S, m_cap), z(S, m_cap), z(S, n_cap)
        self.v, self.goal, self.vbar = z(S, n_cap), z(S, n_cap), z(S, n_cap)
        self.tau, self.taubar = z(S, window, n_cap), z(S, window, n_cap)
        self.a0, self.aref, self.abar = z(S, n_cap), z(S, m_cap), z(S, n_cap)
        self.arch_a, self.arch_a0 = z(window, S, n_cap), z(window, S, n_cap)
        self.arch_aref, self.arch_fac = z(window, S, m_cap), z(window, S, ne)
        self.arch_mask = torch.zeros((window, S, m_cap), dtype=torch.uint8, device=dev)
        # the slot table as a packed batch with capacity offsets; live sizes per slot
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
        fo = self.batch.mask_offset()
        self.fac_view = self.sol.state[:S * ne * s].view(dt).view(S, ne)
        self.mask_view = self.sol.state[fo:fo + S * m_cap].view(S, m_cap)
        self.g_a0, self.g_aref = z(S, n_cap), z(S, m_cap)
        # host bookkeeping
        self.phase = np.full(S, -1, dtype=np.int64)   # -1 free; 0..W-1 forward; W..2W-1 backward
        self.req: List[Optional[Request]] = [None] * S
        self.free = deque(range(S))
        self.queue: deque = deque()
        self.finished: List[Request] = []
        self.pool: Optional[RequestPool] = None
        self.results: Dict[int, torch.Tensor] = {}
        self.keep_results = False
        self.max_active = 0

    def attach_pool(self, pool: RequestPool):
        if pool.Mp.shape[1] != self.n_cap or pool.Jp.shape[1] != self.m_cap:
            raise ValueError("pool capacity differs from the engine's")
        self.pool = pool

    def submit(self, req: Request):
        if req.n > self.n_cap or req.m > self.m_cap:
            raise ValueError("request larger than a slot")
        self.queue.append(req)

    def active(self):
        return int(np.sum(self.phase >= 0))

    # ------------------------------------------------------------ launches
    def _launch_groups(self, slots):
        """Split slots into launch groups (path, order, count, nmax, mmax) by the
        planner's class rules, so a request runs the same kernel instance
        whatever else shares its tick."""
        groups: Dict[tuple, List[int]] = {}
        for s in slots:
            n, m = int(self.nv_host[s]), int(self.nr_host[s])
            fam = batching.default_family(self.dtype, n, m)
            if fam == N.PATH_SMALL:
                key = (fam, batching.n_bucket(n), batching.m_bucket(m))
            else:
                key = (fam, 0 if n <= 32 else 1, 0)
            groups.setdefault(key, []).append(s)
        out = []
        for key in sorted(groups):
            idx = np.asarray(groups[key], dtype=np.int32)
            nmax, mmax = int(self.nv_host[idx].max()), int(self.nr_host[idx].max())
            if key[0] == N.PATH_SMALL:      # compile-time sizes follow the bucket, not the mix
                nmax, mmax = max(nmax, min(key[1], self.n_cap)), max(mmax, min(key[2], self.m_cap))
            out.append((key[0], torch.from_numpy(idx).to(self.device), len(idx), nmax, mmax))
        return out

    def _desc(self, path, idx_dev, count, nmax, mmax):
        d = N.CsBatch()
        C.memmove(C.byref(d), C.byref(self.batch.desc), C.sizeof(N.CsBatch))
        d.order = idx_dev.data_ptr()
        d.count = count
        d.path = path
        d.nv_max, d.nrows_max = nmax, mmax
        return d

    # ------------------------------------------------------------ a tick
    def _admit(self, now):
        adm = []
        while self.queue and self.free and self.queue[0].arrival <= now:
            r = self.queue.popleft()
            s = self.free.popleft()
            r.admitted = now
            self.req[s] = r
            self.phase[s] = 0
            self.nv_host[s], self.nr_host[s] = r.n, r.m
            adm.append((s, r.pool_index))
        if adm:
            slots = np.array([a[0] for a in adm])
            sl = torch.from_numpy(slots).to(self.device)
            pi = torch.tensor([a[1] for a in adm], device=self.device)
            P = self.pool
            self.Mt[sl], self.Jt[sl] = P.Mt[pi], P.Jt[pi]
            self.Minv[sl], self.Jp[sl] = P.Minv[pi], P.Jp[pi]
            self.D[sl], self.pen[sl], self.nmask[sl] = P.D[pi], P.pen[pi], P.nmask[pi]
            self.v[sl], self.goal[sl], self.tau[sl] = P.v0[pi], P.goal[pi], P.tau[pi]
            self.vbar[sl] = 0.0
            self.taubar[sl] = 0.0
            self.nv_dev[sl] = torch.from_numpy(self.nv_host[slots]).to(self.device)
            self.nr_dev[sl] = torch.from_numpy(self.nr_host[slots]).to(self.device)
        self.max_active = max(self.max_active, self.active())
        return len(adm)

    def tick(self, now):
        """Admit, then one batched backward and one batched forward step."""
        self._admit(now)
        W, h = self.W, self.h
        vp, st = solver._vp, solver._stream(self.device)
        bwd = np.flatnonzero(self.phase >= W)
        fwd = np.flatnonzero((self.phase >= 0) & (self.phase < W))
        if len(bwd):     # backward step t = 2W - 1 - phase
            tb = torch.from_numpy(2 * W - 1 - self.phase[bwd]).to(self.device)
            sb = torch.from_numpy(bwd).to(self.device)
            self.sol.a[sb] = self.arch_a[tb, sb]
            self.a0[sb] = self.arch_a0[tb, sb]
            self.aref[sb] = self.arch_aref[tb, sb]
            self.fac_view[sb] = self.arch_fac[tb, sb]
            self.mask_view[sb] = self.arch_mask[tb, sb]
            self.abar[sb] = h * self.vbar[sb]
            for path, od, cnt, nmax, mmax in self._launch_groups(bwd):
                d = self._desc(path, od, cnt, nmax, mmax)
                rc = N.ift_vjp(d, vp(self.sol.state), self.sol.state.numel(), vp(self.Mt),
                               vp(self.Jt), vp(self.a0), vp(self.aref), vp(self.D), vp(self.sol.a),
                               vp(self.abar), vp(self.g_a0), vp(self.g_aref), None, None, None, st)
                N.check(rc, "cs_ift_vjp(serve)")
            nm = self.nmask[sb]
            a0b = self.g_a0[sb] * nm
            arefb = self.g_aref[sb] * (self.D[sb] != 0).to(self.dtype)
            # tau-bar_t = M^-T a0-bar ; v-bar_t = v-bar_{t+1} - b J^T aref-bar
            self.taubar[sb, tb] = torch.bmm(self.Minv[sb].transpose(1, 2).contiguous(),
                                            a0b.unsqueeze(-1)).squeeze(-1) * nm
            self.vbar[sb] = self.vbar[sb] - synth.B_DAMP * torch.bmm(
                self.Jp[sb].transpose(1, 2).contiguous(), arefb.unsqueeze(-1)).squeeze(-1)
        if len(fwd):     # forward step t = phase
            tf = torch.from_numpy(self.phase[fwd]).to(self.device)
            sf = torch.from_numpy(fwd).to(self.device)
            self.a0[sf] = torch.bmm(self.Minv[sf], self.tau[sf, tf].unsqueeze(-1)).squeeze(-1) * self.nmask[sf]
            self.aref[sf] = (-synth.B_DAMP * torch.bmm(self.Jp[sf], self.v[sf].unsqueeze(-1)).squeeze(-1)
                             - synth.K_SPRING * self.pen[sf])
            p = N.CsSolverParams(int(self.max_iter), 0, float(self.tol))
            for path, od, cnt, nmax, mmax in self._launch_groups(fwd):
                d = self._desc(path, od, cnt, nmax, mmax)
                rc = N.forward(d, p, vp(self.Mt), vp(self.Jt), vp(self.a0), vp(self.aref),
                               vp(self.D), None, vp(self.sol.a), vp(self.sol.state),
                               self.sol.state.numel(), vp(self.sol.status), vp(self.sol.iters), st)
                N.check(rc, "cs_forward(serve)")
            a = self.sol.a[sf] * self.nmask[sf]
            self.arch_a[tf, sf] = a
            self.arch_a0[tf, sf] = self.a0[sf]
            self.arch_aref[tf, sf] = self.aref[sf]
            self.arch_fac[tf, sf] = self.fac_view[sf]
            self.arch_mask[tf, sf] = self.mask_view[sf]
            self.v[sf] = self.v[sf] + h * a
        done = np.zeros(0, dtype=np.int64)
        if len(fwd):
            self.phase[fwd] += 1
            last = fwd[self.phase[fwd] == W]
            if len(last):
                sl = torch.from_numpy(last).to(self.device)
                self.vbar[sl] = 2.0 * (self.v[sl] - self.goal[sl])
        if len(bwd):
            self.phase[bwd] += 1
            done = bwd[self.phase[bwd] == 2 * W]
        for s in done:
            r = self.req[s]
            if self.keep_results:
                n = r.n
                self.results[r.rid] = torch.cat([self.v[s, :n], self.taubar[s, :, :n].reshape(-1)]).clone()
            self.req[s] = None
            self.phase[s] = -1
            self.free.append(s)
            self.finished.append(r)
        return len(fwd) + len(bwd), done


def run_stream(engine: Engine, rate, n_requests, warmup=0, seed=0):
    """Serve a Poisson stream of ``rate`` requests/s on the wall clock.

    The host synchronises after every tick, so a request completes when the
    GPU work of its last tick has finished.  Returns latency percentiles (after
    the warm-up requests), throughput in requests and solves per second."""
    rng = np.random.default_rng(seed)
    total = n_requests + warmup
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=total))
    P = engine.pool
    pick = rng.integers(0, len(P.n), size=total)
    reqs = [Request(rid=i, pool_index=int(pick[i]), n=int(P.n[pick[i]]), m=int(P.m[pick[i]]),
                    arrival=float(arrivals[i])) for i in range(total)]
    pending = deque(reqs)
    engine.finished.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solves = ticks = 0
    while len(engine.finished) < total:
        now = time.perf_counter() - t0
        while pending and pending[0].arrival <= now:
            engine.submit(pending.popleft())
        if engine.active() == 0 and not engine.queue:
            if pending:
                time.sleep(max(0.0, min(pending[0].arrival - now, 0.001)))
            continue
        n_work, done = engine.tick(now)
        torch.cuda.synchronize()
        tnow = time.perf_counter() - t0
        for r in engine.finished[len(engine.finished) - len(done):]:
            r.done = tnow
        solves += n_work
        ticks += 1
    elapsed = time.perf_counter() - t0
    fin = sorted(engine.finished, key=lambda r: r.rid)[warmup:]
    lat = np.array([r.done - r.arrival for r in fin])
    span = max(r.done for r in fin) - min(r.arrival for r in fin)
    return dict(rate=rate, requests=len(fin), p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3), requests_per_s=len(fin) / span,
                solves_per_s=solves / elapsed, ticks=ticks, slots=engine.S,
                max_active=engine.max_active)
