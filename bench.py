#!/usr/bin/env python3
"""Throughput benchmark: batched contact solve + IFT VJP on one MI355X.

One step = cs_forward + cs_ift_vjp over one batch of B = 4096 instances with
nv = 9 and 16 contacts (64 pyramid rows), FP32, Newton cap K = 10, tol 1e-5,
inputs resident in HBM.  Steps rotate over enough distinct batches (seeded
synthetic inputs) that their working set exceeds twice the 256 MB last-level
(MALL) cache.  Prints one JSON line.

The throughput comes from one replay of a HIP graph of the K steps in which
each batch's VJP runs on a second stream, overlapping the next batch's
forward (--no-overlap: a graph of the K steps one launch after another; both
step times are reported).  An eager sequential pass over the same K steps
with HIP events around every launch gives the per-kernel durations behind
the dominant kernel's roofline position.  Also measured
(reported inside the same line): the unrolled-trace gradient at the same K on
the same GPU (the library's fused trace kernels, and plain reverse-mode AD of
the same solve by PyTorch autograd), the state/tape memory, and the FP64
oracle timed on the host cores on a bounded sample.
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
MALL_BYTES = 256 * 2 ** 20
HBM_PEAK = 8.0e12          # B/s
FP32_VEC_PEAK = 157.3e12   # flop/s (256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 (dual issue) x 2.4 GHz)


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
    """The FP64 oracle (unmodified) on the FP32-rounded inputs of one batch."""
    import oracle
    b64 = b32.astype(np.float64)
    P = oracle.Packed.uniform(b64.M, b64.J, b64.a0, b64.aref, b64.D, b64.abar)
    threads = oracle.max_threads()
    done, t0 = 0, time.perf_counter()
    reps = 0
    while True:
        fw = P.forward(max_iter=K_CAP, tol=1e-10, threads=threads)
        P.ift_vjp(fw["a"], fw["active"], threads=threads)
        done += P.B
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return dict(value=done / el, unit="solves/s", cores=threads, kind="oracle",
                sample=f"{reps} passes of forward + IFT VJP over one B={B} batch (FP64 oracle on "
                       f"the FP32-rounded inputs, {threads} OpenMP threads, {el:.1f} s)")


def k_sweep(bufs, batch, steps=30):
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
                                        K=K, tol=TOL, tape=tape)
            for i in range(3):
                run(i)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for i in range(steps):
                run(i)
            e1.record()
            torch.cuda.synchronize()
            row[f"{mode}_ms"] = e0.elapsed_time(e1) / steps
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
    sol, grads = plan.capture(t, max_iter=K_CAP, tol=TOL)
    for _ in range(2):
        plan.graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    n = pb.nv.astype(np.float64)
    m = pb.nrows.astype(np.float64)
    byt = float(np.sum([sum(algorithmic_bytes(a, b)) for a, b in zip(n, m)]))
    st = sol.status.cpu().numpy()
    return {"workload": "packed B=8192, nv in {3,9,18,36,96}, contacts U{0..256}, FP32, K=10",
            "ms_per_batch": ms, "solves_per_s": 8192 / (ms / 1e3),
            "gbps_algorithmic": byt / (ms / 1e3) / 1e9, "bytes_per_batch": byt,
            "converged_frac": float(np.mean(st & 1)), "classes": plan.summary(),
            "table": os.path.basename(batching.TABLE_PATH) if os.path.exists(batching.TABLE_PATH) else None,
            "generation_s": round(gen_s, 1)}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-unrolled", action="store_true")
    ap.add_argument("--no-ad", action="store_true", help="skip the plain unrolled-AD comparison")
    ap.add_argument("--no-overlap", action="store_true",
                    help="time the throughput pass with forward and VJP one after another")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the K sweep, the uneven batch and the serving streams")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM-counter calibration)")
    ap.add_argument("--section", choices=("uneven", "serving"),
                    help="only run this workload (for profiling) and print its JSON")
    ap.add_argument("--serve-rates", default="2000,5000,10000,20000,50000")
    ap.add_argument("--serve-requests", type=int, default=10000)
    args = ap.parse_args()
    rates = tuple(int(x) for x in args.serve_rates.split(","))
    if args.section == "uneven":
        print(json.dumps(uneven(reps=5)), flush=True)
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
    per_batch = (B * 4 * (NV * NV * 2 + M_ROWS * NV * 2 + NV * 4 + M_ROWS * 4)
                 + solver.Batch.uniform(B, NV, M_ROWS, torch.float32, device="cpu").state_bytes())
    R = max(8, math.ceil(2 * MALL_BYTES / per_batch) + 1)
    host = make_batches(R, 20260725)
    batch = solver.Batch.uniform(B, NV, M_ROWS, torch.float32, device=dev)
    keys = ("M", "J", "a0", "aref", "D", "abar")
    bufs = []
    for hb in host:
        t = {k: torch.from_numpy(np.ascontiguousarray(getattr(hb, k))).to(dev) for k in keys}
        sol = solver.forward(batch, t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=K_CAP, tol=TOL)
        grads = solver.ift_vjp(batch, sol, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"])
        bufs.append((t, sol, grads))
    torch.cuda.synchronize()

    def step(i, ev=None):
        t, sol, grads = bufs[i % R]
        if ev is not None:
            ev[0].record()
        solver.forward(batch, t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=K_CAP, tol=TOL,
                       out=sol)
        if ev is not None:
            ev[1].record()
        solver.ift_vjp(batch, sol, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"], out=grads)
        if ev is not None:
            ev[2].record()

    # The timed steps run from HIP graphs (one capture of all K steps), so the
    # host's per-call argument checks stay out of the timed region.  In the
    # pipelined graph each batch's VJP runs on a second stream once its
    # forward has finished, overlapping the next batch's forward; the
    # forward that next rewrites a batch's solution buffer first waits for
    # that batch's previous VJP.  Every step is still one forward + one VJP
    # over one batch.
    def capture(pipelined):
        g = torch.cuda.CUDAGraph()
        cap, side = torch.cuda.Stream(), torch.cuda.Stream()   # default priority
        ev_f = [torch.cuda.Event() for _ in range(args.steps)]
        ev_v = [None] * R
        cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cap), torch.cuda.graph(g, stream=cap):
            side.wait_stream(cap)
            for i in range(args.steps):
                j = i % R
                t, sol, grads = bufs[j]
                if pipelined and ev_v[j] is not None:
                    cap.wait_event(ev_v[j])
                solver.forward(batch, t["M"], t["J"], t["a0"], t["aref"], t["D"],
                               max_iter=K_CAP, tol=TOL, out=sol)
                if not pipelined:
                    solver.ift_vjp(batch, sol, t["M"], t["J"], t["a0"], t["aref"], t["D"],
                                   t["abar"], out=grads)
                    continue
                ev_f[i].record(cap)
                side.wait_event(ev_f[i])
                with torch.cuda.stream(side):
                    solver.ift_vjp(batch, sol, t["M"], t["J"], t["a0"], t["aref"], t["D"],
                                   t["abar"], out=grads)
                ev_v[j] = torch.cuda.Event()
                ev_v[j].record(side)
            cap.wait_stream(side)
        torch.cuda.current_stream().wait_stream(cap)
        torch.cuda.synchronize()
        return g

    def timed(g):
        """One replay of a K-step graph; returns (wall ms, GPU ms)."""
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g0.record()
        g.replay()
        g1.record()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3, g0.elapsed_time(g1)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    graphs = {"sequential": capture(False)}
    if not args.no_overlap:
        graphs["pipelined"] = capture(True)
    for g in graphs.values():   # first replay uploads the graph; untimed
        g.replay()
    torch.cuda.synchronize()
    # timed region 1 (the throughput): the K pipelined steps, or the K
    # sequential steps with --no-overlap (the profiled configuration: there
    # every kernel runs alone, so its traced duration is its own)
    wall_seq, gpu_seq = timed(graphs["sequential"])
    if args.no_overlap:
        wall, gpu_ms = wall_seq, gpu_seq
    else:
        wall, gpu_ms = timed(graphs["pipelined"])
    ms = max(wall, gpu_ms)
    value = B * args.steps / (ms / 1e3)
    # timed region 2 (the per-kernel durations for the roofline): the same K
    # steps with HIP events around every launch, on the launch stream
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(args.steps):
        step(i, evs[i])
    torch.cuda.synchronize()
    wall_ev = time.perf_counter() - t1
    progress(f"headline: {value:.4g} solves/s ({ms / args.steps * 1e3:.1f} us per step)")
    t_fwd = np.array([e[0].elapsed_time(e[1]) for e in evs])
    t_vjp = np.array([e[1].elapsed_time(e[2]) for e in evs])

    # convergence / active-set statistics of the benchmarked solves (one batch)
    st = bufs[0][1].status.cpu().numpy()
    it = bufs[0][1].iters.cpu().numpy()
    sb = batch.state_bytes()
    act = batch.active_sets(bufs[0][1]).reshape(B, M_ROWS).sum(1)
    flops_per_launch = float(np.sum(forward_flops(NV, M_ROWS, act, it)))
    fwd_s = float(np.mean(t_fwd)) / 1e3
    vjp_s = float(np.mean(t_vjp)) / 1e3
    fwd_flops_rate = flops_per_launch / fwd_s
    vjp_gbps = B * vjp_b / vjp_s

    out = {
        "metric": "fwd+IFT-VJP contact solves/sec and GB/s vs unrolled-AD; p50/p99 latency",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "timing": {"wall_ms": wall, "gpu_ms": gpu_ms, "overlap": not args.no_overlap,
                   "sequential_ms_per_step": max(wall_seq, gpu_seq) / args.steps,
                   "instrumented_pass_ms": wall_ev * 1e3,
                   "kernel_sum_ms": float(np.sum(t_fwd) + np.sum(t_vjp)),
                   "note": "value from one replay of a HIP graph of the K steps, each batch's "
                           "VJP overlapping the next batch's forward on a second stream "
                           "(sequential_ms_per_step: a graph of the same K steps one launch "
                           "after another; each graph replayed once untimed first); "
                           "per-kernel durations (kernels, roofline) from an eager sequential "
                           "pass of the same K steps with HIP events around every launch"},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "uniform batch B=4096, nv=9, 16 contacts (64 pyramid rows), FP32, "
                               "forward (Newton cap K=10, tol 1e-5) + IFT VJP",
                   "B": B, "nv": NV, "contacts": NC, "rows": M_ROWS, "K": K_CAP, "tol": TOL,
                   "rotating_batches": R, "working_set_MB": round(R * per_batch / 2 ** 20, 1)},
        "gbps_algorithmic": value * (fwd_b + vjp_b) / 1e9,
        "bytes_per_solve": {"forward": fwd_b, "ift_vjp": vjp_b},
        "kernels": {
            "forward_ms": fwd_s * 1e3, "ift_vjp_ms": vjp_s * 1e3,
            "forward_tflops": fwd_flops_rate / 1e12,
            "ift_vjp_gbps": vjp_gbps / 1e9, "ift_vjp_hbm_frac": vjp_gbps / HBM_PEAK,
        },
        "roofline": {"kernel": "k_forward_small<float,9,4>", "bound": "alu",
                     "achieved": fwd_flops_rate / 1e12, "peak": FP32_VEC_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": fwd_flops_rate / FP32_VEC_PEAK,
                     "traffic": measured_traffic("forward"),
                     "algorithmic_bytes_per_launch": B * fwd_b,
                     "flops_per_launch": flops_per_launch},
        "solver": {"converged_frac": float(np.mean(st & 1)), "mean_iters": float(it.mean()),
                   "mean_active_rows": float(act.mean())},
        "memory": {"state_bytes": sb, "tape_bytes_K10": batch.tape_bytes(K_CAP),
                   "tape_bytes_K1": batch.tape_bytes(1)},
    }

    if not args.no_unrolled:
        t, sol, grads = bufs[0]
        n_u = max(10, args.steps // 10)
        tape = torch.empty(batch.tape_bytes(K_CAP), dtype=torch.uint8, device=dev)
        for i in range(3):
            tt = bufs[i % R][0]
            solver.unrolled_vjp(batch, tt["M"], tt["J"], tt["a0"], tt["aref"], tt["D"], tt["abar"],
                                K=K_CAP, tol=TOL, tape=tape)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(n_u):
            tt = bufs[i % R][0]
            solver.unrolled_vjp(batch, tt["M"], tt["J"], tt["a0"], tt["aref"], tt["D"], tt["abar"],
                                K=K_CAP, tol=TOL, tape=tape)
        e1.record()
        torch.cuda.synchronize()
        u_ms = e0.elapsed_time(e1) / n_u
        u_val = B / (u_ms / 1e3)
        out["unrolled"] = {"value": u_val, "unit": "solves/s", "K": K_CAP, "ms_per_step": u_ms,
                           "ift_over_unrolled": value / u_val}
        if not args.no_ad:
            progress("unrolled kernels done")
            out["unrolled_ad"] = unrolled_ad(bufs, R, value)
            progress("plain unrolled AD done")

    if not args.no_extra:
        out["k_sweep"] = k_sweep(bufs, batch)
        progress("K sweep done")
        out["uneven"] = uneven()
        progress("uneven batch done")
        out["serving"] = serving(rates, n_requests=args.serve_requests,
                                 warmup=max(1, args.serve_requests // 10))
    if not args.no_cpu:
        progress("oracle CPU baseline started")
        out["cpu_baseline"] = cpu_baseline(host[0])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
