"""Shared helpers of the GPU parity tests (HIP path vs FP64 oracle)."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_2607_24959_amd import solver, synth

KEYS = ("M", "J", "a0", "aref", "D")
GKEYS = ("a0", "aref", "J", "D", "M")


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def np64(t):
    return t.detach().to("cpu", torch.float64).numpy()


def gpu_uniform(b: synth.UniformBatch, dtype, max_iter, tol, vjp=True, order=None, path=0,
                method="newton"):
    batch = solver.Batch.uniform(b.B, b.n, b.m, dtype, order=order, path=path)
    t = {k: dev(getattr(b, k), dtype) for k in KEYS + ("abar",)}
    sol = solver.forward(batch, *(t[k] for k in KEYS), max_iter=max_iter, tol=tol, method=method)
    out = dict(a=sol.a, status=sol.status, iters=sol.iters, state=sol.state)
    if vjp:
        g = solver.ift_vjp(batch, sol, *(t[k] for k in KEYS), t["abar"])
        out.update(zip(GKEYS, g))
    torch.cuda.synchronize()
    res = {k: (np64(v) if v.dtype.is_floating_point else v.cpu().numpy()) for k, v in out.items()
           if k != "state"}
    res["active"] = batch.active_sets(sol).reshape(b.B, b.m)
    assert sol.state.numel() >= batch.state_bytes()
    return res


def gpu_unrolled_uniform(b: synth.UniformBatch, dtype, K, tol, path=0):
    batch = solver.Batch.uniform(b.B, b.n, b.m, dtype, path=path)
    t = {k: dev(getattr(b, k), dtype) for k in KEYS + ("abar",)}
    out = solver.unrolled_vjp(batch, *(t[k] for k in KEYS), t["abar"], K=K, tol=tol)
    torch.cuda.synchronize()
    return {k: (np64(v) if isinstance(v, torch.Tensor) and v.dtype.is_floating_point else
                (v.cpu().numpy() if isinstance(v, torch.Tensor) else v)) for k, v in out.items()}


def oracle_uniform(b64: synth.UniformBatch, max_iter, tol, vjp=True):
    P = oracle.Packed.uniform(b64.M, b64.J, b64.a0, b64.aref, b64.D, b64.abar)
    fw = P.forward(max_iter=max_iter, tol=tol)
    out = dict(a=fw["a"].reshape(b64.B, b64.n), status=fw["status"], iters=fw["iters"],
               active=fw["active"][:b64.B * b64.m].reshape(b64.B, b64.m).astype(bool))
    if vjp:
        g = P.ift_vjp(fw["a"], fw["active"])
        out.update(a0=g["a0"], aref=g["aref"], J=g["J"], D=g["D"], M=g["M"])
    return out


def oracle_unrolled_uniform(b64: synth.UniformBatch, K, tol):
    P = oracle.Packed.uniform(b64.M, b64.J, b64.a0, b64.aref, b64.D, b64.abar)
    return P.unrolled_vjp(K=K, tol=tol)


def rel_rows(x, ref, B):
    """Per-instance norm-wise relative error of two [B, ...] arrays."""
    x = np.asarray(x).reshape(B, -1)
    ref = np.asarray(ref).reshape(B, -1)
    num = np.linalg.norm(x - ref, axis=1)
    den = np.maximum(np.linalg.norm(ref, axis=1), 1e-30)
    return num / den


def margins(b64: synth.UniformBatch, a):
    """Relative distance of each row's residual from the cone boundary at a."""
    a = a.reshape(b64.B, b64.n)
    r = np.einsum("bij,bj->bi", b64.J, a) - b64.aref
    scale = np.abs(b64.aref) + np.einsum("bij,bj->bi", np.abs(b64.J), np.abs(a)) + 1e-300
    return np.abs(r) / scale


# ------------------------------------------------------------------ FP32 rules
#
# Every FP32 instance is checked individually.  The only exclusions are rules
# computed by the oracle alone:
#  * degenerate (R14): the oracle's a* has a row within TAU_DEG (relative) of
#    the cone boundary; the derivative is one-sided there, so such instances
#    are checked on a (and on the VJP at the GPU's own point), not on the
#    end-to-end gradients;
#  * FP32-ill-conditioned outputs: replacing a* by its FP32 rounding moves the
#    oracle's eq. 17 cotangent X by more than TAU_SENS (relative); no FP32
#    result can then be held to 1e-3, and X is checked against
#    SENS_FACTOR times that movement instead.
# Both fractions are printed and must stay below 1 %.

TAU_DEG = 1e-7
TAU_SENS = 2e-4
SENS_FACTOR = 10.0
TOL_A32, TOL_G32 = 1e-4, 1e-3
TOL_SAMEPT32 = 1e-5


def _few(flags):
    """An excluded set is small: under 1 % of a batch (at most two instances of
    a batch under 200)."""
    flags = np.asarray(flags, bool)
    return flags.mean() < 0.01 if flags.size >= 200 else flags.sum() <= 2


def gpu_packed(pb, dtype, max_iter, tol, path=0, plan=False, vjp=True, method="newton"):
    """Forward (+ IFT VJP) of a packed batch through the C ABI; flat host arrays."""
    from paper_2607_24959_amd import batching
    npd = np.float32 if dtype == torch.float32 else np.float64
    px = pb.astype(npd)
    batch = solver.Batch.packed_from(pb.nv, pb.nrows, dtype, path=path)
    t = {k: dev(getattr(px, k), dtype) for k in KEYS + ("abar",)}
    runner = batching.Plan(batch) if plan else None
    if runner is not None:
        sol = runner.forward(*(t[k] for k in KEYS), max_iter=max_iter, tol=tol)
        g = runner.ift_vjp(sol, *(t[k] for k in KEYS), t["abar"]) if vjp else None
    else:
        sol = solver.forward(batch, *(t[k] for k in KEYS), max_iter=max_iter, tol=tol,
                             method=method)
        g = solver.ift_vjp(batch, sol, *(t[k] for k in KEYS), t["abar"]) if vjp else None
    torch.cuda.synchronize()
    out = dict(a=np64(sol.a).ravel(), status=sol.status.cpu().numpy(), iters=sol.iters.cpu().numpy(),
               active=batch.active_sets(sol))
    if g is not None:
        out.update({k: np64(x).ravel() for k, x in zip(GKEYS, g)})
    return out


def oracle_packed(pb):
    """Oracle batch of the FP32-rounded packed inputs."""
    p64 = pb.rounded(np.float32)
    return oracle.Packed(pb.nv, pb.nrows, p64.M, p64.J, p64.a0, p64.aref, p64.D, p64.abar)


def seg_rel(x, ref, off):
    """Per-instance norm-wise relative error over packed segments off[i]:off[i+1]."""
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    B = len(off) - 1
    out = np.empty(B)
    for i in range(B):
        s = slice(int(off[i]), int(off[i + 1]))
        out[i] = np.linalg.norm(x[s] - ref[s]) / max(np.linalg.norm(ref[s]), 1e-30)
    return out


def packed_margins(P, a):
    """Per instance: min over rows of |r_i| / (|aref_i| + sum_j |J_ij| |a_j|) (inf if no rows)."""
    out = np.full(P.B, np.inf)
    for i in range(P.B):
        n, m = int(P.nv[i]), int(P.nrows[i])
        if m == 0:
            continue
        J = P.J[P.off_mn[i]:P.off_mn[i + 1]].reshape(m, n)
        ar = P.aref[P.off_m[i]:P.off_m[i + 1]]
        ai = np.asarray(a)[P.off_n[i]:P.off_n[i + 1]]
        r = J @ ai - ar
        out[i] = (np.abs(r) / (np.abs(ar) + np.abs(J) @ np.abs(ai) + 1e-300)).min()
    return out


def grad_offsets(P):
    return dict(a0=P.off_n, aref=P.off_m, J=P.off_mn, D=P.off_m, M=P.off_nn)


def packed_from_uniform(b):
    return oracle.Packed.uniform(b.M, b.J, b.a0, b.aref, b.D, b.abar)


def check_fp32(label, P, g, max_iter=60, all_converge=True, fw=None, edge_shapes=False):
    """FP32 GPU results g (a, status, active, and the five gradients, flat) for the
    packed oracle batch P (FP32-rounded inputs in FP64), instance by instance.
    Returns the dict of printed figures."""
    if fw is None:
        fw = P.forward(max_iter=max_iter, tol=1e-10)
    offs = grad_offsets(P)
    B = P.B
    mg = packed_margins(P, fw["a"])
    deg = mg < TAU_DEG
    st_o = fw["status"]
    st_g = np.asarray(g["status"]).ravel()
    conv = (st_o == oracle.ST_CONVERGED) & ((st_g & oracle.ST_CONVERGED) != 0)
    if all_converge:
        assert np.all(st_o == oracle.ST_CONVERGED), label
        assert np.all((st_g & oracle.ST_CONVERGED) != 0), (label, np.flatnonzero((st_g & 1) == 0)[:5])
    act_g = np.asarray(g["active"]).astype(bool).ravel()
    act_o = fw["active"][:int(P.off_m[-1])].astype(bool)
    act_eq = np.array([np.array_equal(act_g[P.off_m[i]:P.off_m[i + 1]], act_o[P.off_m[i]:P.off_m[i + 1]])
                       for i in range(B)])
    ea = seg_rel(g["a"], fw["a"], P.off_n)
    info = dict(label=label, B=B, degenerate=float(deg.mean()), converged=float(conv.mean()),
                act_mismatch_deg=int((~act_eq & deg).sum()), a_max=float(ea.max()))
    assert _few(deg), info
    assert np.all(act_eq | deg), (info, np.flatnonzero(~act_eq & ~deg)[:5])
    assert ea.max() <= TOL_A32, (info, np.argsort(ea)[-3:])
    keys = [k for k in GKEYS if g.get(k) is not None]
    if keys:
        og = P.ift_vjp(fw["a"], fw["active"])
        osp = P.ift_vjp(np.asarray(g["a"], np.float64).ravel(), act_g.astype(np.uint8))
        ar = fw["a"].astype(np.float32).astype(np.float64)
        osn = P.ift_vjp(ar, fw["active"])
        for k in keys:
            sp = seg_rel(g[k], osp[k], offs[k])
            info[f"{k}_samept"] = float(sp.max())
            assert sp.max() <= TOL_SAMEPT32, (label, k, "same point", sp.max(), int(np.argmax(sp)))
            e = seg_rel(g[k], og[k], offs[k])
            sens = seg_rel(osn[k], og[k], offs[k])
            chk = conv & ~deg
            ill = chk & (sens > TAU_SENS)
            ok = chk & ~ill
            info[f"{k}_max"] = float(e[ok].max()) if ok.any() else 0.0
            info[f"{k}_illcond"] = float(ill.mean())
            if not edge_shapes:
                assert _few(ill), (label, k, ill.mean())
            bad = np.flatnonzero(ok & (e > TOL_G32))
            assert bad.size == 0, (label, k, [(int(i), float(e[i]), float(sens[i])) for i in bad[:5]])
            bad = np.flatnonzero(ill & (e > SENS_FACTOR * sens))
            assert bad.size == 0, (label, k, "ill-conditioned", [(int(i), float(e[i]), float(sens[i])) for i in bad[:5]])
    print(info, flush=True)
    return info


def tape_trace_uniform(tape, B, n, m, K, itemsize=4):
    """(A_k, A'_k) bytes of every instance and step from an unrolled tape
    (uniform batch): arrays [B, K, m] of bool."""
    rec = 2 * n + n * (n + 1) // 2 + 2 * m + 2
    base = (itemsize * K * B * rec + 255) // 256 * 256
    tb = np.asarray(tape)[base: base + K * 2 * B * m].reshape(B, K, 2, m)
    return tb[:, :, 0, :].astype(bool), tb[:, :, 1, :].astype(bool)


def oracle_traces(b64, K, tol):
    """Per instance: the oracle's (iters, A [iters, m], A' [iters, m]) of the K-capped solve."""
    out = []
    for i in range(b64.B):
        tr = oracle.forward(b64.M[i], b64.J[i], b64.a0[i], b64.aref[i], b64.D[i], max_iter=K,
                            tol=tol, trace=True)
        out.append((tr["iters"], tr["A"], tr["Ap"]))
    return out


def input_sensitivity(b64, fn, reps=3, seed=1):
    """Largest relative change of fn's per-instance outputs (dict of [B, ...]) when
    every input entry is scaled by 1 +- 2^-24 (random signs): how far any
    FP32 computation of fn may land from it with a few rounding units of
    backward error."""
    rng = np.random.default_rng(seed)
    u = 2.0 ** -24
    pert = lambda x: x * (1.0 + u * rng.choice([-1.0, 1.0], size=x.shape))
    ref = fn(b64.M, b64.J, b64.a0, b64.aref, b64.D)
    sens = {k: np.zeros(b64.B) for k in ref}
    for _ in range(reps):
        o = fn(pert(b64.M), pert(b64.J), pert(b64.a0), pert(b64.aref), pert(b64.D))
        for k in ref:
            sens[k] = np.maximum(sens[k], rel_rows(o[k], ref[k], b64.B))
    return ref, sens


def oracle_iterate(b64, i, k, tol):
    """The oracle's iterate a_k of instance i (k steps of its own path)."""
    return oracle.forward(b64.M[i], b64.J[i], b64.a0[i], b64.aref[i], b64.D[i], max_iter=k,
                          tol=tol)["a"]


def row_margins(b64, i, a):
    r = b64.J[i] @ a - b64.aref[i]
    return np.abs(r) / (np.abs(b64.aref[i]) + np.abs(b64.J[i]) @ np.abs(a) + 1e-300)


def divergence(b64, i, K, tol, tr, A_g, Ap_g, it_g):
    """Where the GPU trace of instance i first leaves the oracle's: ("A" | "Ap", k,
    min margin of the rows that differ, at the oracle's iterate where that row's
    sign was decided), or ("stop", k, None) when only the step count differs."""
    ko, Ao, Apo = tr
    for k in range(min(ko, it_g)):
        if not np.array_equal(Ao[k], A_g[k]):
            rows = np.flatnonzero(Ao[k] != A_g[k])
            return "A", k, float(row_margins(b64, i, oracle_iterate(b64, i, k, tol))[rows].min())
        if not np.array_equal(Apo[k], Ap_g[k]):
            rows = np.flatnonzero(Apo[k] != Ap_g[k])
            return "Ap", k, float(row_margins(b64, i, oracle_iterate(b64, i, k + 1, tol))[rows].min())
    return "stop", min(ko, it_g), None


def subset(pb, g, idx):
    """The instances idx of packed batch pb and of the GPU results g, re-packed."""
    idx = np.asarray(idx)
    sub = synth.pack([dict(n=int(pb.nv[i]), **{k: v for k, v in pb.get(i).items()
                                               if k in ("M", "J", "a0", "aref", "D", "abar")})
                      for i in idx])
    offs = dict(a=pb.off_n, a0=pb.off_n, aref=pb.off_m, J=pb.off_mn, D=pb.off_m, M=pb.off_nn,
                active=pb.off_m)
    gs = {}
    for k, v in g.items():
        if k in offs:
            o = offs[k]
            gs[k] = np.concatenate([np.asarray(v).ravel()[o[i]:o[i + 1]] for i in idx]) if len(idx) else v[:0]
        else:
            gs[k] = np.asarray(v)[idx]
    return sub, gs


U32 = 2.0 ** -24
SOLVE_FACTOR = 4.0


def solve_cond_bound(b64, K, tol):
    """Per instance: u * sum_k kappa_2(H_k) over the Newton matrices of the
    oracle's K-capped trace (u = 2^-24) -- the classical forward-error bound of
    the FP32 solves that a trace derivative passes through."""
    out = np.zeros(b64.B)
    for i in range(b64.B):
        tr = oracle.forward(b64.M[i], b64.J[i], b64.a0[i], b64.aref[i], b64.D[i], max_iter=K,
                            tol=tol, trace=True)
        s = 0.0
        for k in range(tr["iters"]):
            H = b64.M[i] + b64.J[i].T @ ((b64.D[i] * tr["A"][k])[:, None] * b64.J[i])
            s += np.linalg.cond(H)
        out[i] = U32 * s
    return out
