"""Autotuner for the uneven-batch planner: which kernel family runs each tile class.

For every (dtype, padded n, row bucket) class that a workload's shape
distribution produces, it builds a seeded synthetic batch of that class
(the class's largest n and rows drawn uniformly inside the bucket), times
cs_forward + cs_ift_vjp for every family that supports the shape, and keeps
the fastest per instance.  The result is a JSON table that batching.Plan
reads (``families``: key -> CS_PATH_*), together with the measured times.

Run on the GPU:  python -m paper_2607_24959_amd.autotune [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import _native as N
from . import batching, solver, synth

FAMILIES = (N.PATH_SMALL, N.PATH_WAVE, N.PATH_CHUNK, N.PATH_TEAM)


def class_keys(nv_choices, nc_max):
    """Tile classes of a workload with nv drawn from nv_choices and contacts
    from U{0..nc_max}: (padded n, largest n, row bucket, rows in the bucket)."""
    out = []
    for n in sorted(set(nv_choices)):
        nb = batching.n_bucket(n)
        buckets = {}
        for nc in range(nc_max + 1):
            m = synth.ROWS_PER_CONTACT * nc
            buckets.setdefault(batching.m_bucket(m), []).append(m)
        for mb, ms in sorted(buckets.items()):
            out.append((nb, n, mb, ms))
    return out


def _time_family(batch, t, path, max_iter, tol, reps):
    b = solver.Batch.uniform(batch.B, batch.n, batch.m, batch.dtype, device=batch.device, path=path)
    try:
        sol = solver.forward(b, t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=max_iter, tol=tol)
        grads = solver.ift_vjp(b, sol, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"])
    except N.CsError as e:
        if e.code == N.CS_EUNSUPPORTED:
            return None
        raise
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        solver.forward(b, t["M"], t["J"], t["a0"], t["aref"], t["D"], max_iter=max_iter, tol=tol, out=sol)
        solver.ift_vjp(b, sol, t["M"], t["J"], t["a0"], t["aref"], t["D"], t["abar"], out=grads)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps / batch.B * 1e3      # microseconds per instance


def tune(dtype=torch.float32, nv_choices=(3, 9, 18, 36, 96), nc_max=256, B=512, max_iter=10,
         tol=1e-5, reps=5, seed=20260801, log=print):
    npd = np.float32 if dtype == torch.float32 else np.float64
    families, times = {}, {}
    for k, (nb, n, mb, ms) in enumerate(class_keys(nv_choices, nc_max)):
        m = max(ms)
        nc = m // synth.ROWS_PER_CONTACT
        hb = synth.uniform_batch(B, n, nc, seed + k).astype(npd)
        batch = solver.Batch.uniform(B, n, m, dtype, device="cuda")
        t = {key: torch.from_numpy(np.ascontiguousarray(getattr(hb, key))).to("cuda", dtype)
             for key in ("M", "J", "a0", "aref", "D", "abar")}
        res = {}
        for path in FAMILIES:
            us = _time_family(batch, t, path, max_iter, tol, reps)
            if us is not None:
                res[path] = us
        best = min(res, key=res.get)
        key = batching.table_key(dtype, nb, mb)
        families[key] = int(best)
        times[key] = {str(p): round(v, 4) for p, v in res.items()}
        log(f"{key}: n={n} m={m} " + " ".join(f"path{p}={v:.3f}us" for p, v in res.items())
            + f" -> path{best}")
    return families, times


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=batching.TABLE_PATH)
    ap.add_argument("--B", type=int, default=512)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("the autotuner times kernels and needs a GPU")
    t0 = time.time()
    fam, times = {}, {}
    for dt in (torch.float32, torch.float64):
        f, tm = tune(dtype=dt, B=args.B, reps=args.reps)
        fam.update(f)
        times.update(tm)
    meta = {"device": torch.cuda.get_device_name(0), "B": args.B, "reps": args.reps,
            "max_iter": 10, "workload": "nv in {3,9,18,36,96}, contacts U{0..256}",
            "seconds": round(time.time() - t0, 1)}
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump({"families": fam, "us_per_instance": times, "meta": meta}, f, indent=1, sort_keys=True)
    print(f"wrote {args.out} ({len(fam)} classes, {meta['seconds']} s)", flush=True)


if __name__ == "__main__":
    main()
