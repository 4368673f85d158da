"""Semi-implicit rollout through the differentiable contact solve.

Each step solves the contact problem for the acceleration and integrates
v_{t+1} = v_t + h a_t.  The smooth model around the solve is minimal: the
unconstrained acceleration is a0_t = M^{-1} tau_t (Sec. III-A, eq. 1 with no
bias force) and the reference acceleration of each pyramid row follows the
spring-damper rule aref = -b J v_t - k pen used for the synthetic
instances, so the gradient w.r.t. tau flows through a0 (and through aref via
v_t) at every step.
"""
from __future__ import annotations

import torch

from . import _native as N
from . import solver, synth
from .autograd import contact_solve


def rollout(M, J, D, pen, v0, tau, *, h=0.002, max_iter=50, tol=None, backward="ift",
            batch=None, path=0, collect=None):
    """Roll out len(tau) steps.  Shapes: M [B,n,n], J [B,m,n], D [B,m], pen [B,nc],
    v0 [B,n], tau [T,B,n].  Returns v_T.  ``collect`` (a list) receives each
    step's (a, status)."""
    Minv = torch.linalg.inv(M)
    pen_rows = torch.repeat_interleave(pen, synth.ROWS_PER_CONTACT, dim=-1)
    v = v0
    for t in range(tau.shape[0]):
        a0 = torch.bmm(Minv, tau[t].unsqueeze(-1)).squeeze(-1)
        aref = -synth.B_DAMP * torch.bmm(J, v.unsqueeze(-1)).squeeze(-1) - synth.K_SPRING * pen_rows
        a, st = contact_solve(M, J, a0, aref, D, max_iter=max_iter, tol=tol, backward=backward,
                              batch=batch, path=path, return_status=True)
        if collect is not None:
            collect.append((a.detach(), st))
        v = v + h * a
    return v


def make_rollout_problem(B, n, nc, horizon, seed, dtype=torch.float64, device="cuda"):
    """Synthetic rollout workload: instance geometry from the generator, then
    v0, v_goal ~ N(0, 1) and tau_t ~ N(0, 1) from the same seeded stream."""
    import numpy as np
    b = synth.uniform_batch(B, n, nc, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    v0 = rng.standard_normal((B, n))
    v_goal = rng.standard_normal((B, n))
    tau = rng.standard_normal((horizon, B, n))
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(device, dtype)
    return dict(M=t(b.M), J=t(b.J), D=t(b.D), pen=t(b.pen), v0=t(v0), v_goal=t(v_goal), tau=t(tau))


def step_jacobians(M, J, D, sol, batch, h=0.002):
    """iLQR's linearised contact dynamics of one semi-implicit step at the
    solution `sol` of that step (forward-mode IFT, eq. 15): with
    v_{t+1} = v_t + h a*(a0 = M^{-1} tau_t, aref = -b J v_t - k pen),
      B_t = d v_{t+1} / d tau_t = h H^{-1}       (directions M^{-1} e_j of a0),
      A_t = d v_{t+1} / d v_t = I + h H^{-1} J^T D_A (-b J)
                                                 (directions -b J e_j of aref),
    all 2n columns from one cs_ift_jvp call.  Shapes M [B,n,n], J [B,m,n],
    D [B,m]; returns (A_t, B_t), each [B, n, n]."""
    Bn, m, n = J.shape
    Minv = torch.linalg.inv(M)
    da0 = torch.zeros(Bn, 2 * n, n, dtype=M.dtype, device=M.device)
    daref = torch.zeros(Bn, 2 * n, m, dtype=M.dtype, device=M.device)
    da0[:, :n, :] = Minv.transpose(1, 2)                    # row j: column j of M^{-1}
    daref[:, n:, :] = (-synth.B_DAMP * J).transpose(1, 2)   # row j: -b J e_j
    da = solver.ift_jvp(batch, sol, M.contiguous(), J.contiguous(), D.contiguous(), 2 * n,
                        da0.reshape(-1), daref.reshape(-1)).reshape(Bn, 2 * n, n)
    eye = torch.eye(n, dtype=M.dtype, device=M.device).expand(Bn, n, n)
    B_t = h * da[:, :n, :].transpose(1, 2)
    A_t = eye + h * da[:, n:, :].transpose(1, 2)
    return A_t, B_t


# ------------------------------------------------------------------ fused rollout
#
# The same rollout as `rollout`, forward and backward each in one launch of
# cs_rollout (J, M and M's factor stay on chip for the whole horizon).

def _fused_call(batch, flags, max_iter, tol, h, M, J, D, c, v0, tau, v_goal=None, vbar_T=None,
                ws=None, status=None, iters=None, v_T=None, recompute=False):
    T_h = tau.shape[0]
    p = N.CsRolloutParams(int(T_h), int(flags | (N.ROLLOUT_RECOMPUTE if recompute else 0)),
                          int(max_iter), 0, float(tol), float(h), float(synth.B_DAMP))
    need = N.rollout_workspace_bytes(batch.desc, p)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=M.device)
    if status is None:
        status = torch.empty(batch.B, dtype=torch.int32, device=M.device)
    if iters is None:
        iters = torch.empty(batch.B, dtype=torch.int32, device=M.device)
    fwd, bwd = bool(flags & N.ROLLOUT_FORWARD), bool(flags & N.ROLLOUT_BACKWARD)
    if fwd and v_T is None:
        v_T = torch.empty_like(v0)
    tau_bar = torch.empty_like(tau) if bwd else None
    v0_bar = torch.empty(batch.B, M.shape[-1], dtype=M.dtype, device=M.device) if bwd else None
    vp = solver._vp
    rc = N.rollout(batch.desc, p, vp(M), vp(J), vp(D), vp(c), vp(v0), vp(tau), vp(v_goal),
                   vp(vbar_T), vp(v_T), vp(tau_bar), vp(v0_bar), vp(ws), ws.numel(), vp(status),
                   vp(iters), solver._stream(M.device))
    N.check(rc, "cs_rollout")
    return dict(v_T=v_T, tau_bar=tau_bar, v0_bar=v0_bar, ws=ws, status=status, iters=iters)


def _fused_inputs(M, J, D, pen, v0, tau):
    B, m, n = J.shape
    c = (-synth.K_SPRING * torch.repeat_interleave(pen, synth.ROWS_PER_CONTACT, dim=-1)).contiguous()
    batch = solver.Batch.uniform(B, n, m, M.dtype, device=M.device)
    return batch, M.contiguous(), J.contiguous(), D.contiguous(), c, v0.contiguous(), tau.contiguous()


def _default_tol(dtype):
    return 1e-12 if dtype == torch.float64 else 1e-5


class _FusedRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, M, J, D, pen, v0, tau, h, max_iter, tol, recompute):
        batch, Mc, Jc, Dc, c, v0c, tauc = _fused_inputs(M, J, D, pen, v0, tau)
        out = _fused_call(batch, N.ROLLOUT_FORWARD, max_iter, tol, h, Mc, Jc, Dc, c, v0c, tauc,
                          recompute=recompute)
        ctx.batch, ctx.args = batch, (max_iter, tol, h, recompute)
        ctx.save_for_backward(Mc, Jc, Dc, c, tauc, out["ws"], out["status"])
        ctx.mark_non_differentiable(out["status"])
        return out["v_T"], out["status"]

    @staticmethod
    def backward(ctx, gv, _gst):
        Mc, Jc, Dc, c, tauc, ws, status = ctx.saved_tensors
        max_iter, tol, h, recompute = ctx.args
        out = _fused_call(ctx.batch, N.ROLLOUT_BACKWARD, max_iter, tol, h, Mc, Jc, Dc, c, None, tauc,
                          vbar_T=gv.contiguous(), ws=ws, status=status, recompute=recompute)
        return None, None, None, None, out["v0_bar"], out["tau_bar"], None, None, None, None


def fused_rollout(M, J, D, pen, v0, tau, *, h=0.002, max_iter=50, tol=None, recompute=False):
    """v_T of the rollout `rollout` computes, from one cs_rollout launch; its
    backward (w.r.t. tau and v0) is one more launch.  Returns (v_T, status)."""
    tol = _default_tol(M.dtype) if tol is None else tol
    return _FusedRollout.apply(M, J, D, pen, v0, tau, float(h), int(max_iter), float(tol),
                               bool(recompute))


def fused_loss_grad(M, J, D, pen, v0, tau, v_goal, *, h=0.002, max_iter=50, tol=None,
                    recompute=False):
    """Forward, loss ||v_T - v_goal||^2 and its gradient w.r.t. tau and v0 in
    ONE launch.  Returns dict(v_T, tau_bar, v0_bar, status, iters)."""
    tol = _default_tol(M.dtype) if tol is None else tol
    batch, Mc, Jc, Dc, c, v0c, tauc = _fused_inputs(M, J, D, pen, v0, tau)
    return _fused_call(batch, N.ROLLOUT_FORWARD | N.ROLLOUT_BACKWARD, max_iter, tol, h, Mc, Jc, Dc,
                       c, v0c, tauc, v_goal=v_goal.contiguous(), recompute=recompute)
