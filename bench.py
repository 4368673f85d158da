#!/usr/bin/env python3
"""Throughput benchmark: batched contact solve + IFT VJP on one MI355X.

One step = cs_forward + cs_ift_vjp over one batch of B = 4096 instances with
nv = 9 and 16 contacts (64 pyramid rows), FP32, Newton cap K = 10, tol 1e-5,
inputs resident in HBM.  Steps rotate over enough distinct batches (seeded
synthetic inputs) that their working set exceeds twice the 256 MB last-level
(MALL) cache.  Prints one JSON line.

The K timed steps are captured once into a HIP graph; the value is the median
over 20 timed replays of that graph (each replay exactly K steps, bracketed by
synchronisation; one untimed replay first), in the fastest of three schedules
(one stream; each VJP on a second stream overlapping the next forward; two
independent chains of batches on two streams).  Graphs of the K forwards
alone and of the K VJPs alone, timed the same way, give the per-kernel
durations behind the dominant kernel's roofline position.

Also in the same line: the same workload with a cap (K = 40) at which every
instance converges, so the IFT is evaluated at the tolerance-converged root
the paper's derivative is defined at; the FP64 path at the same shape; the
nonlinear-CG forward feeding the same VJP; the unrolled-trace gradient at
K = 10 (the library's fused trace kernels, timed from a graph like the IFT
path, and plain reverse-mode AD of the same solve by PyTorch autograd); the K
sweep with memory; the uneven batch; the iLQR step Jacobians; the fused
rollout gradient; the serving streams; and the FP64 oracle timed on the host
cores on bounded samples.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

B, NV, NC = 4096, 9, 16
M_ROWS = 4 * NC
K_CAP, TOL = 10, 1e-5
K_CONV = 40               # cap at which every instance of the workload converges
MALL_BYTES = 256 * 2 ** 20
HBM_PEAK = 8.0e12          # B/s
FP32_VEC_PEAK = 157.3e12   # flop/s (256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 (dual issue) x 2.4 GHz)
FP64_VEC_PEAK = 78.6e12    # flop/s (256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz)


def progress(msg):
    """One line on stderr as each part of the run finishes."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(n, m, s=4):
    """Compulsory HBM traffic per solve of cs_forward and cs_ift_vjp (all outputs)."""
    fwd = s * (n * n + m * n + n + 2 * m) + s * n + math.ceil(m / 8)
    vjp = s * (3 * n + n * n + m * n + 2 * m) + math.ceil(m / 8) + s * (n + 2 * m + m * n + n * n)
    return fwd, vjp


def forward_flops(n, m, active, iters):
    """Algorithmic flops of one forward solve.

    Per Newton step: r = J a - aref (2mn), F = M(a-a0) + J^T w (2n^2 + 2mn),
    H = M + J^T D_A J on the lower triangle (|A| n (n+1)), Cholesky (n^3/3),
    solve (2n^2), q = J p (2mn), line-search coefficients (4n^2), two
    line-search passes over the rows (8m) and the update (2n).  The returned
    iterate adds one residual/gradient/Hessian/Cholesky evaluation.
    """
    step = 8 * m * n + 8 * n * n + active * n * (n + 1) + n ** 3 / 3 + 8 * m + 2 * n
    final = 4 * m * n + 2 * n * n + active * n * (n + 1) + n ** 3 / 3
    return iters * step + final


def fp64_roofline(kernel, flops, ms):
    """Roofline position of an FP64-arithmetic kernel: algorithmic flops of one
    launch over its duration, against the FP64 vector peak."""
    rate = flops / (ms / 1e3)
    return {"kernel": kernel, "bound": "alu", "achieved": rate / 1e12, "peak": FP64_VEC_PEAK / 1e12,
            "unit": "TFLOP/s", "frac": rate / FP64_VEC_PEAK, "flops_per_launch": flops}


def ell_flops(n, nc, live, iters, ls_evals=5.3):
    """Algorithmic flops of one round-cone forward: per Newton step the
    pyramid model's row passes over m = 3 nc rows, K = G J for the live
    contacts (18 n each), H over their 3 rows (3 live n (n+1)), the Cholesky,
    and ls_evals line-search evaluations of every contact's block (~60 flops)."""
    m = 3 * nc
    step = 8 * m * n + 8 * n * n + 18 * live * n + 3 * live * n * (n + 1) + n ** 3 / 3 + \
        ls_evals * 60 * nc + 2 * n
    return iters * step + 4 * m * n + 2 * n * n + 3 * live * n * (n + 1) + n ** 3 / 3


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_uniform_B4096_n9_m64.txt")


def measured_traffic(key="forward"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel sources have changed since the counters were taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals, srcs = {}, []
    for line in open(TRAFFIC_FILE):
        line = line.strip()
        if " = " in line:
            k, v = line.split(" = ", 1)
            vals[k] = v
        elif line.startswith("paper_2607_24959_amd/csrc/"):
            srcs.append(line)
    h = hashlib.sha256()
    for f in srcs:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if not srcs or vals.get("sources_sha256") != h.hexdigest():
        return None
    v = vals.get(f"traffic_bytes.{key}")
    return int(v) if v is not None else None


def make_batches(count, seed0):
    from paper_2607_24959_amd import synth
    return [synth.uniform_batch(B, NV, NC, seed0 + i).astype(np.float32) for i in range(count)]


def cpu_baseline(b32, seconds=10.0):
    """The FP64 oracle (unmodified) on the FP32-rounded inputs of one batch,
    on all host threads; also on one thread, and on a stratified sample of the
    uneven batch."""
    import oracle
    from paper_2607_24959_amd import synth
    b64 = b32.astype(np.float64)
    P = oracle.Packed.uniform(b64.M, b64.J, b64.a0, b64.aref, b64.D, b64.abar)

    def rate(P, threads, seconds):
        done, reps, t0 = 0, 0, time.perf_counter()
        while True:
            fw = P.forward(max_iter=K_CAP, tol=1e-10, threads=threads)
            P.ift_vjp(fw["a"], fw["active"], threads=threads)
            done += P.B
            reps += 1
            el = time.perf_counter() - t0
            if el >= seconds:
                return done / el, reps, el

    threads = oracle.max_threads()
    v, reps, el = rate(P, threads, seconds)
    v1, reps1, el1 = rate(P, 1, seconds / 3)
    # the uneven batch: 82 instances of every nv (5 % of B = 8192), same seed
    pb = synth.uneven_batch(8192, (3, 9, 18, 36, 96), 256, seed=synth.SEED_BASE + 2)
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.choice(np.flatnonzero(pb.nv == n), 82, replace=False)
                          for n in (3, 9, 18, 36, 96)])
    sub = synth.pack([dict(n=int(pb.nv[i]), **{k: x for k, x in pb.get(i).items()
                                               if k in ("M", "J", "a0", "aref", "D", "abar")})
                      for i in idx]).rounded(np.float32)
    Pu = oracle.Packed(sub.nv, sub.nrows, sub.M, sub.J, sub.a0, sub.aref, sub.D, sub.abar)
    vu, repsu, elu = rate(Pu, threads, 0.0)
    return dict(value=v, unit="solves/s", cores=threads, kind="oracle",
                sample=f"{reps} passes of forward + IFT VJP over one B={B} batch (FP64 oracle on "
                       f"the FP32-rounded inputs, {threads} OpenMP threads, {el:.1f} s)",
                one_core={"value": v1, "unit": "solves/s",
                          "sample": f"{reps1} passes, 1 thread, {el1:.1f} s"},
                uneven_sample={"value": vu, "unit": "solves/s", "instances": int(idx.size),
                               "ms_per_B8192_batch_scaled": 8192 / vu * 1e3,
                               "sample": "stratified 5 % of the uneven batch (82 instances of "
                                         f"every nv), forward cap 10 + IFT VJP, {threads} threads, "
                                         f"{elu:.1f} s"})


def k_sweep(bufs, batch, steps=20):
    """IFT (forward at cap K + VJP) against the unrolled trace at K = 1..10:
    time per batch and the temporary device memory of each gradient path."""
    import torch
    from paper_2607_24959_amd import solver
    R = len(bufs)
    tape = torch.empty(batch.tape_bytes(10), dtype=torch.uint8, device="cuda")
    out = []
    for K in range(1, 11):
        row = {"K": K}
        for mode in ("ift", "unrolled"):
            def run(i, mode=mode, K=K):
                t, sol, grads = bufs[i % R]
                if mode == "ift":
                    solver.forward(batch, t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=K, tol=TOL,
                                   out=sol)
                    solver.ift_vjp(batch, sol, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"],
                                   out=grads)
                else:
                    solver.unrolled_vjp(batch, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"],
                                        K=K, tol=TOL, tape=tape, out=uouts[i % R])
            if mode == "unrolled":
                uouts = [solver.unrolled_vjp(batch, b[0]["M"], b[0]["J"], b[0]["a0"], b[0]["aref"],
                                             b[0]["D"], b[0]["abar"], K=K, tol=TOL, tape=tape)
                         for b in bufs]
            for i in range(3):
                run(i)
            torch.cuda.synchronize()
            # both paths timed alike: a graph of `steps` steps on one stream
            g = torch.cuda.CUDAGraph()
            cap = torch.cuda.Stream()
            cap.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(cap), torch.cuda.graph(g, stream=cap):
                for i in range(steps):
                    run(i)
            torch.cuda.current_stream().wait_stream(cap)
            torch.cuda.synchronize()
            ms, _ = replay_median(g, reps=5)
            del g
            row[f"{mode}_ms"] = ms / steps
            # peak temporary memory of one fresh call (outputs allocated by the call)
            torch.cuda.synchronize()
            base = torch.cuda.memory_allocated()
            torch.cuda.reset_peak_memory_stats()
            t = bufs[0][0]
            if mode == "ift":
                sol = solver.forward(batch, t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=K, tol=TOL)
                g = solver.ift_vjp(batch, sol, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"])
            else:
                g = solver.unrolled_vjp(batch, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"],
                                        K=K, tol=TOL)
            torch.cuda.synchronize()
            row[f"{mode}_peak_bytes"] = torch.cuda.max_memory_allocated() - base
            del g
        row["state_bytes"] = batch.state_bytes()
        row["tape_bytes"] = batch.tape_bytes(K)
        row["ift_over_unrolled"] = row["unrolled_ms"] / row["ift_ms"]
        out.append(row)
    return out


def unrolled_ad(bufs, R, ift_value, reps=3):
    """Plain unrolled reverse-mode AD of the same K-step solve: PyTorch autograd
    through the batched tensor program (eager), on the same batches.  Time per
    gradient of the whole batch, and the peak memory it holds at K=1 and K=10."""
    import torch
    from paper_2607_24959_amd import ad_unrolled

    def call(t, K=K_CAP):
        return ad_unrolled.vjp(t["M"].reshape(B, NV, NV), t["J"].reshape(B, M_ROWS, NV),
                               t["a0"].reshape(B, NV), t["aref"].reshape(B, M_ROWS),
                               t["D"].reshape(B, M_ROWS), t["abar"].reshape(B, NV), K=K, tol=TOL)

    peaks = {}
    for K in (1, K_CAP):
        call(bufs[0][0], K)
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        call(bufs[0][0], K)
        torch.cuda.synchronize()
        peaks[K] = torch.cuda.max_memory_allocated() - base
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(reps):
        call(bufs[i % R][0])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    val = B / (ms / 1e3)
    return {"what": "PyTorch autograd through the same batched K-step solve (eager tensor ops)",
            "value": val, "unit": "solves/s", "K": K_CAP, "ms_per_step": ms,
            "ift_over_unrolled_ad": ift_value / val,
            "peak_bytes_K1": peaks[1], f"peak_bytes_K{K_CAP}": peaks[K_CAP]}


def uneven(reps=20):
    """B=8192 packed instances, nv in {3,9,18,36,96}, contacts U{0..256}, FP32:
    tile classes from the autotuned table, LPT order, forward + IFT VJP of all
    classes captured in one HIP graph and replayed."""
    import torch
    from paper_2607_24959_amd import batching, solver, synth
    t0 = time.perf_counter()
    pb = synth.uneven_batch(8192, (3, 9, 18, 36, 96), 256, seed=synth.SEED_BASE + 2).astype(np.float32)
    gen_s = time.perf_counter() - t0
    batch = solver.Batch.packed_from(pb.nv, pb.nrows, torch.float32)
    plan = batching.Plan(batch)
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(pb, k))).to("cuda") for k in
         ("M", "J", "a0", "aref", "D", "abar")}
    per = {}
    for lanes in (1, 2):
        sol, grads = plan.capture(t, max_iter=K_CAP, tol=TOL, lanes=lanes)
        per[lanes], _ = replay_median(plan.graph, reps=reps)
        plan.graph = None
    lanes = min(per, key=per.get)
    ms = per[lanes]
    n = pb.nv.astype(np.float64)
    m = pb.nrows.astype(np.float64)
    byt = float(np.sum([sum(algorithmic_bytes(a, b)) for a, b in zip(n, m)]))
    st = sol.status.cpu().numpy()
    return {"workload": "packed B=8192, nv in {3,9,18,36,96}, contacts U{0..256}, FP32, K=10",
            "ms_per_batch": ms, "solves_per_s": 8192 / (ms / 1e3),
            "gbps_algorithmic": byt / (ms / 1e3) / 1e9, "bytes_per_batch": byt,
            "converged_frac": float(np.mean(st & 1)), "classes": plan.summary(),
            "lanes": lanes, "ms_per_batch_by_lanes": per,
            "table": os.path.basename(batching.TABLE_PATH) if os.path.exists(batching.TABLE_PATH) else None,
            "generation_s": round(gen_s, 1)}


def ilqr_jacobians(reps=20):
    """iLQR's linearised contact dynamics for the rollout workload's shape
    (B=1024, nv=18, 32 contacts, FP32): A_t and B_t of one step from one
    cs_ift_jvp call with 2 nv = 36 directions per instance (eq. 15), timed
    from a graph.  Roofline: FP64 vector peak (the kernel computes in FP64);
    flops per direction counted as the two refined solves would need them."""
    import torch
    from paper_2607_24959_amd import solver, synth
    Bn, n, nc = 1024, 18, 32
    m = 4 * nc
    b = synth.uniform_batch(Bn, n, nc, synth.SEED_BASE + 3).astype(np.float32)
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(b, k))).cuda() for k in
         ("M", "J", "a0", "aref", "D")}
    batch = solver.Batch.uniform(Bn, n, m, torch.float32)
    sol = solver.forward(batch, t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=K_CONV, tol=TOL)
    k = 2 * n
    rng = np.random.default_rng(0)
    da0 = torch.from_numpy(rng.standard_normal(k * Bn * n).astype(np.float32)).cuda()
    daref = torch.from_numpy(rng.standard_normal(k * Bn * m).astype(np.float32)).cuda()
    out = solver.ift_jvp(batch, sol, t["M"], t["J"], t["D"], k, da0, daref)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap), torch.cuda.graph(g, stream=cap):
        for _ in range(10):
            solver.ift_jvp(batch, sol, t["M"], t["J"], t["D"], k, da0, daref, out=out)
    torch.cuda.current_stream().wait_stream(cap)
    torch.cuda.synchronize()
    ms, spread = replay_median(g, reps=reps)
    ms /= 10
    act = batch.active_sets(sol).reshape(Bn, m).sum(1).astype(np.float64)
    # per direction: rhs (2 n^2 + 4 |A| n) and, three times, a solve (2 n^2)
    # plus (for the two refinements) H x (2 n^2 + 4 |A| n)
    per_dir = 3 * (2 * n * n + 4 * act * n) + 3 * 2 * n * n
    flops = float(np.sum(per_dir) * k)
    return {"workload": f"B={Bn}, nv={n}, {nc} contacts, FP32, {k} directions per instance "
                        "(the A_t and B_t columns of one step)",
            "ms_per_batch": ms, "jacobian_columns_per_s": Bn * k / (ms / 1e3),
            "replay_spread": spread,
            "roofline": {"bound": "alu", "achieved": flops / (ms / 1e3) / 1e12, "peak": 78.6,
                         "unit": "TFLOP/s (FP64 vector)", "frac": flops / (ms / 1e3) / 78.6e12}}


def ell_line(steps=20, K=40, tol=1e-5):
    """The round (elliptic) cone at the headline's shape: B=4096, nv=9, 16
    contacts (48 rows: normal + two tangential per contact), FP32 storage
    (FP64 arithmetic), cap K=40 at which every instance converges, forward +
    IFT VJP; rotating batches over twice the MALL, a graph of `steps` steps,
    median of replays; per-kernel times from graphs of one kernel kind."""
    import torch
    from paper_2607_24959_amd import solver, synth
    nc, m = NC, 3 * NC
    batch = solver.Batch.uniform(B, NV, m, torch.float32)
    per_batch = B * 4 * (NV * NV + m * NV + 2 * NV + m + 3 * nc) + batch.state_bytes()
    R = max(8, math.ceil(2 * MALL_BYTES / per_batch) + 1)
    R += R % 2
    keys = ("M", "J", "a0", "aref", "dn", "dt", "mu")
    bufs = []
    for r in range(R):
        eb = synth.elliptic_batch(B, NV, nc, 20260725 + 500 + r).astype(np.float32)
        t = {k: torch.from_numpy(np.ascontiguousarray(getattr(eb, k))).cuda()
             for k in keys + ("abar",)}
        sol = solver.forward_ell(batch, *(t[k] for k in keys), max_iter=K, tol=tol)
        gr = solver.ift_vjp_ell(batch, sol, *(t[k] for k in keys), t["abar"])
        bufs.append((t, sol, gr))
    torch.cuda.synchronize()

    def fwd(t, sol, gr):
        solver.forward_ell(batch, *(t[k] for k in keys), max_iter=K, tol=tol, out=sol)

    def vjp(t, sol, gr):
        solver.ift_vjp_ell(batch, sol, *(t[k] for k in keys), t["abar"], out=gr)

    def graph(fns):
        g = torch.cuda.CUDAGraph()
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st), torch.cuda.graph(g, stream=st):
            for i in range(steps):
                for fn in fns:
                    fn(*bufs[i % R])
        torch.cuda.current_stream().wait_stream(st)
        torch.cuda.synchronize()
        return g, st

    g, st = graph((fwd, vjp))
    ms, spread = replay_median(g)
    gf, sf = graph((fwd,))
    t_f = replay_median(gf)[0] / steps
    gv, sv = graph((vjp,))
    t_v = replay_median(gv)[0] / steps
    stat = np.concatenate([b[1].status.cpu().numpy() for b in bufs[:steps]])
    its = np.concatenate([b[1].iters.cpu().numpy() for b in bufs[:steps]])
    z = batch.zones(bufs[0][1])
    live = (z.reshape(B, nc) != 0).sum(1)
    it0 = bufs[0][1].iters.cpu().numpy()
    flops = float(np.sum(ell_flops(NV, nc, live, it0)))
    del g, gf, gv, st, sf, sv
    return {"roofline": fp64_roofline("k_forward_ell<float>", flops, t_f),
            "workload": f"round cone, uniform batch B={B}, nv={NV}, {nc} contacts ({m} rows), "
                        f"FP32 storage (FP64 arithmetic), cap K={K}, tol {tol}, forward + IFT VJP",
            "value": B * steps / (ms / 1e3), "unit": "solves/s", "ms_per_step": ms / steps,
            "replay_spread": spread, "rotating_batches": R,
            "kernels": {"forward_ms": t_f, "ift_vjp_ms": t_v},
            "solver": {"converged_frac": float(np.mean((stat & 1) != 0)),
                       "lsfail_count": int(np.sum((stat & 16) != 0)),
                       "mean_iters": float(its.mean()), "max_iters": int(its.max()),
                       "zone_fractions": [float(np.mean(z == k)) for k in (0, 1, 2)]}}


def rows_line(steps=20, K=40, tol=1e-5, ne=4, nf=8):
    """Mixed rows at the headline's shape: B=4096, nv=9, 16 contacts (64
    pyramid rows) plus 4 equality and 8 friction-loss rows, FP32 storage (FP64
    arithmetic), cap K=40, forward + IFT VJP; timed like ell_line."""
    import torch
    from paper_2607_24959_amd import solver, synth
    m = 4 * NC + ne + nf
    batch = solver.Batch.uniform(B, NV, m, torch.float32)
    per_batch = B * (4 * (NV * NV + m * NV + 2 * NV + 3 * m) + m) + batch.state_bytes()
    R = max(8, math.ceil(2 * MALL_BYTES / per_batch) + 1)
    R += R % 2
    keys = ("M", "J", "a0", "aref", "D")
    bufs = []
    for r in range(R):
        mb = synth.mixed_batch(B, NV, NC, ne, nf, 20260725 + 700 + r).astype(np.float32)
        t = {k: torch.from_numpy(np.ascontiguousarray(getattr(mb, k))).cuda()
             for k in keys + ("floss", "abar")}
        t["kind"] = torch.from_numpy(np.ascontiguousarray(mb.kind)).cuda()
        sol = solver.forward_rows(batch, *(t[k] for k in keys), t["kind"], t["floss"], max_iter=K,
                                  tol=tol)
        gr = solver.ift_vjp_rows(batch, sol, *(t[k] for k in keys), t["kind"], t["floss"], t["abar"])
        bufs.append((t, sol, gr))
    torch.cuda.synchronize()

    def fwd(t, sol, gr):
        solver.forward_rows(batch, *(t[k] for k in keys), t["kind"], t["floss"], max_iter=K, tol=tol,
                            out=sol)

    def vjp(t, sol, gr):
        solver.ift_vjp_rows(batch, sol, *(t[k] for k in keys), t["kind"], t["floss"], t["abar"],
                            out=gr)

    def graph(fns):
        g = torch.cuda.CUDAGraph()
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st), torch.cuda.graph(g, stream=st):
            for i in range(steps):
                for fn in fns:
                    fn(*bufs[i % R])
        torch.cuda.current_stream().wait_stream(st)
        torch.cuda.synchronize()
        return g, st

    g, st = graph((fwd, vjp))
    ms, spread = replay_median(g)
    gf, sf = graph((fwd,))
    t_f = replay_median(gf)[0] / steps
    gv, sv = graph((vjp,))
    t_v = replay_median(gv)[0] / steps
    stat = np.concatenate([b[1].status.cpu().numpy() for b in bufs[:steps]])
    its = np.concatenate([b[1].iters.cpu().numpy() for b in bufs[:steps]])
    o = batch.mask_offset()
    zone0 = bufs[0][1].state[o:o + B * m].cpu().numpy().reshape(B, m)
    flops = float(np.sum(forward_flops(NV, m, (zone0 == 1).sum(1), bufs[0][1].iters.cpu().numpy())))
    del g, gf, gv, st, sf, sv
    return {"roofline": fp64_roofline("k_forward_rows<float>", flops, t_f),
            "workload": f"mixed rows, uniform batch B={B}, nv={NV}, {NC} contacts ({4 * NC} pyramid "
                        f"rows) + {ne} equality + {nf} friction-loss rows, FP32 storage (FP64 "
                        f"arithmetic), cap K={K}, tol {tol}, forward + IFT VJP",
            "value": B * steps / (ms / 1e3), "unit": "solves/s", "ms_per_step": ms / steps,
            "replay_spread": spread, "rotating_batches": R,
            "kernels": {"forward_ms": t_f, "ift_vjp_ms": t_v},
            "solver": {"converged_frac": float(np.mean((stat & 1) != 0)),
                       "lsfail_count": int(np.sum((stat & 16) != 0)),
                       "mean_iters": float(its.mean()), "max_iters": int(its.max())}}


def rollout_line(B_=1024, n=18, nc=32, horizon=50, reps=5):
    """The differentiation workload (B=1024, nv=18, 32 contacts, h=0.002,
    horizon 50, FP64, loss ||v_T - v_goal||^2): the gradient w.r.t. tau by
    the fused rollout (forward and backward through time in one cs_rollout
    launch; keeping each step's factor, or recomputing it) against the
    layered rollout (one forward launch per step, autograd backward with one
    IFT VJP launch per step).  Median of `reps` timed runs each (HIP events,
    one untimed run first)."""
    import torch
    from paper_2607_24959_amd import rollout as R
    P = R.make_rollout_problem(B_, n, nc, horizon, seed=20260727)

    def fused(recompute):
        return lambda: R.fused_loss_grad(P["M"], P["J"], P["D"], P["pen"], P["v0"], P["tau"],
                                         P["v_goal"], max_iter=60, tol=1e-12, recompute=recompute)

    def layered():
        tau = P["tau"].clone().requires_grad_(True)
        v = R.rollout(P["M"], P["J"], P["D"], P["pen"], P["v0"], tau, max_iter=60, tol=1e-12)
        ((v - P["v_goal"]) ** 2).sum().backward()
        return tau.grad

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0.record()
            out = fn()
            e1.record()
            torch.cuda.synchronize()
            ms.append(max(e0.elapsed_time(e1), (time.perf_counter() - t0) * 1e3))
        return float(np.median(ms)), out

    t_store, o = timed(fused(False))
    t_rec, _ = timed(fused(True))
    t_lay, g_lay = timed(layered)
    e = ((o["tau_bar"] - g_lay).transpose(0, 1).flatten(1).norm(dim=1) /
         g_lay.transpose(0, 1).flatten(1).norm(dim=1)).max().item()
    # algorithmic flops of the fused launch: every Newton step of every solve
    # (forward_flops at the step's average active-row count, read from the
    # workspace's saved active sets) plus the backward per step (a solve with
    # the kept factor, J lambda and J^T s: 4 n^2 + 4 m n)
    m = 4 * nc
    step_bytes = o["ws"].numel() // horizon
    masks = o["ws"].view(horizon, step_bytes)[:, step_bytes - ((B_ * m + 255) // 256 * 256):]
    act = masks[:, :B_ * m].reshape(horizon, B_, m).sum(-1).double().mean(0).cpu().numpy()
    its = o["iters"].double().cpu().numpy()
    final = 4 * m * n + 2 * n * n + act * n * (n + 1) + n ** 3 / 3
    flops = float(np.sum(forward_flops(n, m, act, its) + (horizon - 1) * final +
                         horizon * (4 * n * n + 4 * m * n)))
    return {"roofline": fp64_roofline("k_rollout<double>", flops, t_store),
            "workload": f"rollout gradient, B={B_}, nv={n}, {nc} contacts, horizon {horizon}, "
                        "h=0.002, FP64, tol 1e-12",
            "fused_ms": t_store, "fused_recompute_ms": t_rec, "layered_ms": t_lay,
            "fused_speedup": t_lay / t_store,
            "rollouts_per_s": B_ / (t_store / 1e3),
            "newton_steps_per_solve": float(o["iters"].double().mean().item()) / horizon,
            "converged_frac": float(((o["status"] & 1) != 0).double().mean().item()),
            "lsfail_count": int(((o["status"] & 16) != 0).sum().item()),
            "max_rel_diff_vs_layered": e}


def serving(rates=(2000, 5000, 10000, 20000, 50000), n_requests=10000, warmup=1000,
            budget_bytes=256 * 2 ** 20):
    """Poisson streams of 6-step MPC windows (nv in {3,9,18}, contacts U{0..64},
    FP32, Newton cap 10), slots from an HBM budget."""
    import torch
    from paper_2607_24959_amd import serve
    pool = serve.RequestPool(4096, (3, 9, 18), 64, 6, 20260802, 18, 256, torch.float32, "cuda")
    out = []
    for rate in rates:
        eng = serve.Engine(budget_bytes=budget_bytes, window=6, max_iter=K_CAP, tol=TOL)
        eng.attach_pool(pool)
        r = serve.run_stream(eng, rate=float(rate), n_requests=n_requests, warmup=warmup, seed=rate)
        r["budget_MiB"] = budget_bytes / 2 ** 20
        out.append(r)
        del eng
    return out


N_REPLAYS = 20
CG_CAPS = (600, 20000)   # CG steps are heavy-tailed: a practical cap, and one where all converge


SCHEDULES = ("sequential", "vjp_overlap", "two_chains")


def capture_steps(bufs, batch, steps, K, tol, schedule, method="newton"):
    """HIP graph of `steps` steps (forward at cap K + IFT VJP, batch i % R at
    step i), in one of three schedules:
      sequential  -- one stream, one launch after another;
      vjp_overlap -- forwards on one stream, each VJP on a second once its
                     forward is done (overlapping the next batch's forward); a
                     forward that rewrites a batch's solution first waits for
                     that batch's previous VJP;
      two_chains  -- step i on stream i % 2 (R is even, so a batch always runs
                     on the same stream and no event is needed): two
                     independent chains of batches share the device.
    Returns (graph, keep): every stream and event the capture used is in
    `keep`, alive as long as the graph."""
    import torch
    from paper_2607_24959_amd import solver
    R = len(bufs)
    assert schedule != "two_chains" or R % 2 == 0
    g = torch.cuda.CUDAGraph()
    nst = 1 if schedule == "sequential" else 2
    streams = [torch.cuda.Stream() for _ in range(nst)]     # default priority
    keep = {"streams": streams, "events": []}
    cap = streams[0]
    cap.wait_stream(torch.cuda.current_stream())
    last_vjp = [None] * R
    with torch.cuda.stream(cap), torch.cuda.graph(g, stream=cap):
        for st in streams[1:]:
            st.wait_stream(cap)
        for i in range(steps):
            j = i % R
            t, sol, grads = bufs[j]
            if schedule == "two_chains":
                fl = vl = streams[i % 2]
            elif schedule == "vjp_overlap":
                fl, vl = cap, streams[1]
            else:
                fl = vl = cap
            if last_vjp[j] is not None:
                fl.wait_event(last_vjp[j])
            with torch.cuda.stream(fl):
                solver.forward(batch, t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=K,
                               tol=tol, out=sol, method=method)
            if vl is not fl:
                ef = torch.cuda.Event()
                ef.record(fl)
                keep["events"].append(ef)
                vl.wait_event(ef)
            with torch.cuda.stream(vl):
                solver.ift_vjp(batch, sol, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"],
                               out=grads)
            if vl is not fl:
                ev = torch.cuda.Event()
                ev.record(vl)
                keep["events"].append(ev)
                last_vjp[j] = ev
        for st in streams[1:]:
            cap.wait_stream(st)
    torch.cuda.current_stream().wait_stream(cap)
    torch.cuda.synchronize()
    return g, keep


def replay_median(g, reps=N_REPLAYS):
    """Median over `reps` timed replays (one untimed first) of max(GPU ms by
    HIP events, host wall ms), each replay bracketed by synchronisation."""
    import torch
    g.replay()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        out.append(max((time.perf_counter() - t0) * 1e3, e0.elapsed_time(e1)))
    out = np.array(out)
    return float(np.median(out)), {"min_ms": float(out.min()), "max_ms": float(out.max()),
                                   "replays": reps}


def kernel_times(bufs, batch, steps, K, tol, method="newton"):
    """Per-kernel durations on the launch stream: one HIP graph of the `steps`
    forwards alone (back to back on one stream) and one of the `steps` IFT
    VJPs alone, each timed like the throughput line (HIP events around the
    replay, median of replays); the mean launch is the replay time / steps.
    Leaves batches 0 .. steps-1 solved at cap K."""
    import torch
    from paper_2607_24959_amd import solver
    R = len(bufs)

    def graph(fn):
        g = torch.cuda.CUDAGraph()
        st = torch.cuda.Stream()   # default priority
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st), torch.cuda.graph(g, stream=st):
            for i in range(steps):
                fn(*bufs[i % R])
        torch.cuda.current_stream().wait_stream(st)
        torch.cuda.synchronize()
        return g, st

    gf, sf = graph(lambda t, sol, grads: solver.forward(
        batch, t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=K, tol=tol, out=sol,
        method=method))
    t_fwd = replay_median(gf)[0] / steps
    gv, sv = graph(lambda t, sol, grads: solver.ift_vjp(
        batch, sol, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"], out=grads))
    t_vjp = replay_median(gv)[0] / steps
    del gf, gv, sf, sv
    return t_fwd, t_vjp


def solve_stats(bufs, batch, B_, m):
    """Convergence, iterations, active rows and line-search safeguard hits over
    every rotating batch (as the last pass left them)."""
    st = np.concatenate([b[1].status.cpu().numpy() for b in bufs])
    it = np.concatenate([b[1].iters.cpu().numpy() for b in bufs])
    act0 = batch.active_sets(bufs[0][1]).reshape(B_, m).sum(1)
    return {"converged_frac": float(np.mean(st & 1)), "mean_iters": float(it.mean()),
            "max_iters": int(it.max()), "lsfail_count": int(np.sum((st & 16) != 0)),
            "instances": int(st.size), "mean_active_rows": float(act0.mean())}, act0, \
        bufs[0][1].iters.cpu().numpy()


def make_bufs(host, batch, dev, K, tol, dtype):
    import torch
    from paper_2607_24959_amd import solver
    keys = ("M", "J", "a0", "aref", "D", "abar")
    bufs = []
    for hb in host:
        t = {k: torch.from_numpy(np.ascontiguousarray(getattr(hb, k))).to(dev, dtype) for k in keys}
        sol = solver.forward(batch, t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=K, tol=tol)
        grads = solver.ift_vjp(batch, sol, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"])
        bufs.append((t, sol, grads))
    torch.cuda.synchronize()
    return bufs


def rotation(s, state_bytes):
    """Rotating batches: at least 8, and more than twice the MALL in total."""
    per_batch = B * s * (NV * NV * 2 + M_ROWS * NV * 2 + NV * 4 + M_ROWS * 4) + state_bytes
    R = max(8, math.ceil(2 * MALL_BYTES / per_batch) + 1)
    return R + (R % 2), per_batch


def ift_line(bufs, batch, steps, K, tol, schedules=SCHEDULES, s=4, method="newton"):
    """One throughput line: a graph of `steps` steps at cap K in each schedule,
    median of replays each; the line's value is the fastest schedule's.  Also
    per-kernel times, solver statistics and the forward's roofline position."""
    per = {}
    for sch in schedules:
        g, keep = capture_steps(bufs, batch, steps, K, tol, sch, method)
        ms_s, spread_s = replay_median(g)
        del g, keep
        per[sch] = {"ms_per_step": ms_s / steps, "replay_spread": spread_s}
    best = min(per, key=lambda k: per[k]["ms_per_step"])
    ms, spread = per[best]["ms_per_step"] * steps, per[best]["replay_spread"]
    t_fwd, t_vjp = kernel_times(bufs, batch, steps, K, tol, method)
    # the forward graph above left batches 0 .. steps-1 solved at cap K
    stats, act, it = solve_stats(bufs[:min(steps, len(bufs))], batch, B, M_ROWS)
    fwd_b, vjp_b = algorithmic_bytes(NV, M_ROWS, s)
    flops = float(np.sum(forward_flops(NV, M_ROWS, act, it)))
    value = B * steps / (ms / 1e3)
    return {"value": value, "ms_per_step": ms / steps, "replay_spread": spread, "schedule": best,
            "schedules_ms_per_step": {k: v["ms_per_step"] for k, v in per.items()},
            "K": K, "tol": tol,
            "kernels": {"forward_ms": t_fwd, "ift_vjp_ms": t_vjp,
                        "forward_tflops": flops / (t_fwd / 1e3) / 1e12,
                        "forward_gbps": B * fwd_b / (t_fwd / 1e3) / 1e9,
                        "ift_vjp_gbps": B * vjp_b / (t_vjp / 1e3) / 1e9,
                        "ift_vjp_hbm_frac": B * vjp_b / (t_vjp / 1e3) / HBM_PEAK,
                        "forward_flops_per_launch": flops},
            "gbps_algorithmic": value * (fwd_b + vjp_b) / 1e9,
            "solver": stats}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-unrolled", action="store_true")
    ap.add_argument("--no-ad", action="store_true", help="skip the plain unrolled-AD comparison")
    ap.add_argument("--schedule", choices=SCHEDULES + ("all",), default="all",
                    help="graph schedule of the timed steps (all: time each, report the fastest)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the converging, FP64, K-sweep, uneven and serving lines")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM-counter calibration)")
    ap.add_argument("--section", choices=("uneven", "serving", "rollout", "elliptic", "rows"),
                    help="only run this workload (for profiling) and print its JSON")
    ap.add_argument("--serve-rates", default="2000,5000,10000,20000,50000")
    ap.add_argument("--serve-requests", type=int, default=10000)
    args = ap.parse_args()
    rates = tuple(int(x) for x in args.serve_rates.split(","))
    if args.section == "uneven":
        print(json.dumps(uneven(reps=5)), flush=True)
        return
    if args.section == "rows":
        print(json.dumps(rows_line(args.steps)), flush=True)
        return
    if args.section == "elliptic":
        print(json.dumps(ell_line(args.steps)), flush=True)
        return
    if args.section == "rollout":
        print(json.dumps(rollout_line(reps=3)), flush=True)
        return
    if args.section == "serving":
        print(json.dumps(serving(rates, n_requests=args.serve_requests,
                                 warmup=max(1, args.serve_requests // 10))), flush=True)
        return
    if args.copy_probe:
        import torch
        n = args.copy_probe * 2 ** 20 // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (instances are "
              "independent, so a multi-GPU run would be B/G instances per GPU at the same "
              "shape)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_24959_amd import solver
    dev = torch.device("cuda:0")

    fwd_b, vjp_b = algorithmic_bytes(NV, M_ROWS)
    batch = solver.Batch.uniform(B, NV, M_ROWS, torch.float32, device=dev)
    R, per_batch = rotation(4, batch.state_bytes())
    host = make_batches(R, 20260725)
    bufs = make_bufs(host, batch, dev, K_CAP, TOL, torch.float32)
    # warm-up: W untimed steps
    for i in range(args.warmup):
        t, sol, grads = bufs[i % R]
        solver.forward(batch, t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=K_CAP, tol=TOL,
                       out=sol)
        solver.ift_vjp(batch, sol, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"], out=grads)
    torch.cuda.synchronize()

    scheds = SCHEDULES if args.schedule == "all" else (args.schedule,)
    head = ift_line(bufs, batch, args.steps, K_CAP, TOL, scheds)
    value = head["value"]
    seq_ms = head["schedules_ms_per_step"].get("sequential")
    progress(f"headline: {value:.4g} solves/s ({head['ms_per_step'] * 1e3:.1f} us per step, "
             f"{head['schedule']}); per schedule (us): "
             + ", ".join(f"{k} {v * 1e3:.1f}" for k, v in head["schedules_ms_per_step"].items()))
    kh = head["kernels"]
    fwd_rate = kh["forward_flops_per_launch"] / (kh["forward_ms"] / 1e3)

    out = {
        "metric": "fwd+IFT-VJP contact solves/sec and GB/s vs unrolled-AD; p50/p99 latency",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "timing": {"replay_spread": head["replay_spread"], "schedule": head["schedule"],
                   "schedules_ms_per_step": head["schedules_ms_per_step"],
                   "note": f"value: median over {N_REPLAYS} timed replays of one HIP graph of "
                           "the K steps (each replay bracketed by synchronisation, max of GPU "
                           "and host time; one untimed replay first), in the fastest of three "
                           "schedules (one stream; VJPs on a second stream overlapping the next "
                           "forward; two independent chains of batches on two streams); "
                           "per-kernel durations from graphs of the forwards alone and of the VJPs "
                           "alone (HIP events around the replay, median of replays, / steps)"},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "uniform batch B=4096, nv=9, 16 contacts (64 pyramid rows), FP32, "
                               "forward (Newton cap K=10, tol 1e-5) + IFT VJP",
                   "B": B, "nv": NV, "contacts": NC, "rows": M_ROWS, "K": K_CAP, "tol": TOL,
                   "rotating_batches": R, "working_set_MB": round(R * per_batch / 2 ** 20, 1)},
        "gbps_algorithmic": head["gbps_algorithmic"],
        "bytes_per_solve": {"forward": fwd_b, "ift_vjp": vjp_b},
        "kernels": kh,
        "roofline": {"kernel": "k_forward_small<float,9,4>", "bound": "alu",
                     "achieved": fwd_rate / 1e12, "peak": FP32_VEC_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": fwd_rate / FP32_VEC_PEAK,
                     "traffic": measured_traffic("forward"),
                     "algorithmic_bytes_per_launch": B * fwd_b,
                     "flops_per_launch": kh["forward_flops_per_launch"],
                     "hbm_frac": B * fwd_b / (kh["forward_ms"] / 1e3) / HBM_PEAK},
        "solver": head["solver"],
        "memory": {"state_bytes": batch.state_bytes(), "tape_bytes_K10": batch.tape_bytes(K_CAP),
                   "tape_bytes_K1": batch.tape_bytes(1)},
    }

    if not args.no_extra:
        # the paper's derivative is defined at the tolerance-converged root:
        # the same workload at a cap where every instance converges
        conv = ift_line(bufs, batch, args.steps, K_CONV, TOL, scheds)
        kc = conv["kernels"]
        rate_c = kc["forward_flops_per_launch"] / (kc["forward_ms"] / 1e3)
        conv["roofline"] = {"kernel": "k_forward_small<float,9,4>", "bound": "alu",
                            "achieved": rate_c / 1e12, "peak": FP32_VEC_PEAK / 1e12,
                            "unit": "TFLOP/s", "frac": rate_c / FP32_VEC_PEAK}
        conv["workload"] = f"as the headline, Newton cap K={K_CONV}"
        out["converged_line"] = conv
        progress(f"converging cap K={K_CONV}: {conv['value']:.4g} solves/s, converged "
                 f"{conv['solver']['converged_frac']:.4f}")
        out["fp64_line"] = fp64_line(args.steps, dev)
        progress("FP64 line done")
        # the other solver for the same minimiser: nonlinear CG forward + the
        # same IFT VJP
        out["cg_lines"] = []
        for cap in CG_CAPS:
            cg = ift_line(bufs, batch, args.steps, cap, TOL, ("sequential",), method="cg")
            del cg["kernels"]["forward_tflops"], cg["kernels"]["forward_flops_per_launch"]
            cg["workload"] = (f"as the headline, nonlinear CG forward (cap {cap} CG steps, "
                              "tol 1e-5) + IFT VJP")
            cg["newton_converged_over_cg"] = conv["value"] / cg["value"]
            out["cg_lines"].append(cg)
            progress(f"CG forward cap {cap}: {cg['value']:.4g} solves/s, converged "
                     f"{cg['solver']['converged_frac']:.4f}, mean CG steps "
                     f"{cg['solver']['mean_iters']:.1f}")
        # back to the headline state for what follows
        for i in range(R):
            t, sol, grads = bufs[i]
            solver.forward(batch, t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=K_CAP,
                           tol=TOL, out=sol)
        torch.cuda.synchronize()

    if not args.no_unrolled:
        u = unrolled_graph(bufs, batch, args.steps)
        u["ift_over_unrolled"] = value / u["value"]
        u["ift_over_unrolled_sequential"] = (B / (seq_ms / 1e3)) / u["value"] if seq_ms else None
        out["unrolled"] = u
        progress("unrolled kernels done")
        if not args.no_ad:
            out["unrolled_ad"] = unrolled_ad(bufs, R, value)
            progress("plain unrolled AD done")

    if not args.no_extra:
        out["k_sweep"] = k_sweep(bufs, batch)
        progress("K sweep done")
        out["uneven"] = uneven()
        progress("uneven batch done")
        out["ilqr_jacobians"] = ilqr_jacobians()
        progress("iLQR Jacobians done")
        out["elliptic"] = ell_line(args.steps)
        progress(f"round cone: {out['elliptic']['value']:.4g} solves/s, converged "
                 f"{out['elliptic']['solver']['converged_frac']:.4f}")
        out["mixed_rows"] = rows_line(args.steps)
        progress(f"mixed rows: {out['mixed_rows']['value']:.4g} solves/s")
        out["rollout"] = rollout_line()
        progress(f"fused rollout: {out['rollout']['fused_ms']:.3g} ms vs layered "
                 f"{out['rollout']['layered_ms']:.3g} ms")
        out["serving"] = serving(rates, n_requests=args.serve_requests,
                                 warmup=max(1, args.serve_requests // 10))
    if not args.no_cpu:
        progress("oracle CPU baseline started")
        out["cpu_baseline"] = cpu_baseline(host[0])
    print(json.dumps(out), flush=True)


def fp64_line(steps, dev):
    """The FP64 path at the headline's shape (the paper computes in FP64):
    cap K=40, tol 1e-10, forward + IFT VJP."""
    import torch
    from paper_2607_24959_amd import _native as N
    from paper_2607_24959_amd import solver, synth
    batch = solver.Batch.uniform(B, NV, M_ROWS, torch.float64, device=dev)
    R, per_batch = rotation(8, batch.state_bytes())
    host = [synth.uniform_batch(B, NV, NC, 20260725 + i) for i in range(R)]
    bufs = make_bufs(host, batch, dev, K_CONV, 1e-10, torch.float64)
    line = ift_line(bufs, batch, steps, K_CONV, 1e-10, ("sequential",), s=8)
    fam = {N.PATH_SMALL: "SMALL", N.PATH_WAVE: "WAVE", N.PATH_CHUNK: "CHUNK",
           N.PATH_TEAM: "TEAM"}
    line["workload"] = (f"uniform batch B={B}, nv={NV}, {NC} contacts, FP64, cap K={K_CONV}, "
                        "tol 1e-10, forward + IFT VJP")
    line["rotating_batches"] = R
    line["working_set_MB"] = round(R * per_batch / 2 ** 20, 1)
    line["family"] = "CHUNK (one 64-lane workgroup per instance)"
    del bufs
    torch.cuda.empty_cache()
    return line


def unrolled_graph(bufs, batch, steps, K=K_CAP):
    """The library's unrolled-trace VJP at cap K over the same rotating batches,
    timed like the IFT path: graphs of `steps` steps (one stream, and two
    independent chains on two streams, each chain with its own tape), median of
    replays, the faster schedule reported."""
    import torch
    from paper_2607_24959_amd import solver
    R = len(bufs)
    tapes = [torch.empty(batch.tape_bytes(K), dtype=torch.uint8, device="cuda") for _ in range(2)]
    outs = []
    for i in range(R):
        t = bufs[i][0]
        outs.append(solver.unrolled_vjp(batch, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"],
                                        K=K, tol=TOL, tape=tapes[i % 2]))
    torch.cuda.synchronize()
    per = {}
    for sch in ("sequential", "two_chains"):
        g = torch.cuda.CUDAGraph()
        streams = [torch.cuda.Stream() for _ in range(1 if sch == "sequential" else 2)]
        cap = streams[0]
        cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cap), torch.cuda.graph(g, stream=cap):
            for st in streams[1:]:
                st.wait_stream(cap)
            for i in range(steps):
                t = bufs[i % R][0]
                with torch.cuda.stream(streams[i % len(streams)]):
                    solver.unrolled_vjp(batch, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"],
                                        K=K, tol=TOL, tape=tapes[i % len(streams)], out=outs[i % R])
            for st in streams[1:]:
                cap.wait_stream(st)
        torch.cuda.current_stream().wait_stream(cap)
        torch.cuda.synchronize()
        ms, spread = replay_median(g)
        del g
        per[sch] = (ms, spread)
    best = min(per, key=lambda k: per[k][0])
    ms, spread = per[best]
    return {"value": B * steps / (ms / 1e3), "unit": "solves/s", "K": K,
            "ms_per_step": ms / steps, "replay_spread": spread, "schedule": best,
            "schedules_ms_per_step": {k: v[0] / steps for k, v in per.items()},
            "what": "fused unrolled-trace kernels (record + reverse sweep, one launch per "
                    "step), HIP graphs timed like the IFT path, median of replays"}


if __name__ == "__main__":
    main()
