"""Differentiable batched contact solve for torch.autograd.

``contact_solve`` returns a* for a batch; its backward is either the IFT
vector-Jacobian product (Sec. III-C, eq. 17: one solve with the saved factor
of H(A*), no solver trace kept) or, for comparison, reverse mode through the
recorded K-step solver trace (the trace is written in the forward pass and
held until the backward pass, like unrolled automatic differentiation).

Every tensor is a device tensor of one dtype; uniform batches use shapes
M [B, n, n], J [B, m, n], a0 [B, n], aref [B, m], D [B, m].
"""
from __future__ import annotations

import torch

from . import solver


class _IFTSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, M, J, a0, aref, D, batch, max_iter, tol):
        sol = solver.forward(batch, M, J, a0, aref, D, max_iter=max_iter, tol=tol)
        ctx.batch = batch
        ctx.sol = sol
        ctx.save_for_backward(M, J, a0, aref, D)
        ctx.mark_non_differentiable(sol.status)
        return sol.a, sol.status

    @staticmethod
    def backward(ctx, abar, _status_bar):
        M, J, a0, aref, D = ctx.saved_tensors
        need = ctx.needs_input_grad
        needs = (need[2], need[3], need[1], need[4], need[0])     # a0, aref, J, D, M
        if abar is None or not any(needs):
            return (None,) * 8
        g = solver.ift_vjp(ctx.batch, ctx.sol, M, J, a0, aref, D, abar.contiguous(), needs=needs)
        a0b, arefb, Jb, Db, Mb = g
        return Mb, Jb, a0b, arefb, Db, None, None, None


class _UnrolledSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, M, J, a0, aref, D, batch, K, tol):
        rec = solver.unrolled_record(batch, M, J, a0, aref, D, K=K, tol=tol)
        ctx.batch = batch
        ctx.rec = rec
        ctx.save_for_backward(M, J, a0, aref, D)
        ctx.mark_non_differentiable(rec["status"])
        return rec["a"], rec["status"]

    @staticmethod
    def backward(ctx, abar, _status_bar):
        M, J, a0, aref, D = ctx.saved_tensors
        need = ctx.needs_input_grad
        needs = (need[2], need[3], need[1], need[4], need[0])
        if abar is None or not any(needs):
            return (None,) * 8
        a0b, arefb, Jb, Db, Mb = solver.unrolled_replay(ctx.batch, ctx.rec, M, J, a0, aref, D,
                                                         abar.contiguous(), needs=needs)
        return Mb, Jb, a0b, arefb, Db, None, None, None


def _batch_for(M, J, batch, path):
    if batch is not None:
        return batch
    B, m, n = J.shape
    return solver.Batch.uniform(B, n, m, M.dtype, device=M.device, path=path)


def contact_solve(M, J, a0, aref, D, *, max_iter=50, tol=None, backward="ift", batch=None,
                  path=0, return_status=False):
    """a* of every instance; differentiable w.r.t. M, J, a0, aref, D.

    backward="ift": cs_ift_vjp at the returned solution (memory independent
    of the number of solver steps).  backward="unrolled": exactly max_iter
    recorded steps, differentiated through the trace (memory grows with it).
    """
    if tol is None:
        tol = 1e-12 if M.dtype == torch.float64 else 1e-5
    M, J, a0, aref, D = (x.contiguous() for x in (M, J, a0, aref, D))
    b = _batch_for(M, J, batch, path)
    if backward == "ift":
        a, st = _IFTSolve.apply(M, J, a0, aref, D, b, int(max_iter), float(tol))
    elif backward == "unrolled":
        a, st = _UnrolledSolve.apply(M, J, a0, aref, D, b, int(max_iter), float(tol))
    else:
        raise ValueError(backward)
    return (a, st) if return_status else a
