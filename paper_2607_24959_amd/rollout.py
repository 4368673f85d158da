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
