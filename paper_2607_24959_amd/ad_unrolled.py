"""Plain unrolled reverse-mode AD: the comparison baseline of the implicit VJP.

The paper compares its implicit derivative (Sec. III-C, eq. 17) with
differentiating the executed K-iteration solver trace by ordinary reverse-mode
automatic differentiation (Sec. V, gradient and memory comparison).  This
module is that baseline on this stack: the same Newton solve -- residual and
active set (eq. 6), Newton matrix (eq. 9), direction, exact line search
(eq. 10), the tolerance stop rule with a cap of K steps -- written in batched
PyTorch tensor operations, with torch.autograd recording every iteration and
reversing it.  It is what a user gets without a hand-written derivative, and
its memory grows with K because autograd keeps each iteration's tensors.

Conventions match the library's unrolled-trace VJP, so both differentiate the
same function: M is used as a general matrix (M (a - a0), H = M + J^T D_A J
solved by LU), the line-search step alpha takes the value the search returns
and the derivative of -b/c on the accepted piece with that piece held fixed,
and steps after the stop rule are the identity.

Comparison only: the solver API (cs_forward / cs_ift_vjp / cs_unrolled_vjp)
never calls this module.
"""
from __future__ import annotations

import math

import torch


def _piece(r, q, D, c0, b0, t):
    """Active rows of phi(t) = L(a + t p) at step t, and the slope c and
    intercept b of phi' = c t + b on that piece."""
    act = (r + t.unsqueeze(-1) * q) < 0
    w = D * act
    return act, c0 + (w * q * q).sum(-1), b0 + (w * q * r).sum(-1)


@torch.no_grad()
def line_search(r, q, D, c0, b0, max_rounds: int = 96):
    """Exact minimiser of the convex piecewise quadratic phi along p (eq. 10)
    by the safeguarded piece-Newton iteration, batched over instances.

    Trial step 1; on each piece, the root -b/c of phi' on that piece is taken
    when it lies inside the current bracket, else bisection (or doubling while
    there is no upper end); the search ends when a Newton point lands on the
    piece that produced it, phi' is exactly zero, or the bracket is below
    32 ulp.  Returns (t, act): the step and the accepted piece's rows.
    """
    eps = torch.finfo(r.dtype).eps
    t = torch.ones(r.shape[0], dtype=r.dtype, device=r.device)
    act, c, b = _piece(r, q, D, c0, b0, t)
    lo = torch.zeros_like(t)
    hi = torch.full_like(t, math.inf)
    done = torch.zeros_like(t, dtype=torch.bool)
    for _ in range(max_rounds):
        gp = c * t + b
        run = ~done
        lo = torch.where(run & (gp < 0), t, lo)
        hi = torch.where(run & (gp >= 0), t, hi)
        done = done | (gp == 0) | (torch.isfinite(hi) & (hi - lo <= 32 * eps * hi))
        if bool(done.all()):
            break
        cand = -b / c
        newton = (cand > lo) & (cand < hi)
        cand = torch.where(newton, cand, torch.where(torch.isfinite(hi), 0.5 * (lo + hi), 2 * lo + 1))
        nact, nc, nb = _piece(r, q, D, c0, b0, cand)
        same = (nact == act).all(-1)
        run = ~done
        act = torch.where(run.unsqueeze(-1), nact, act)
        c = torch.where(run, nc, c)
        b = torch.where(run, nb, b)
        t = torch.where(run, cand, t)
        done = done | (run & newton & same)
    return t, act


def solve(M, J, a0, aref, D, K: int, tol: float, trace=None):
    """a_K of the K-step Newton solve of every instance, differentiable by
    torch.autograd through every iteration.  Shapes: M [B, n, n], J [B, m, n],
    a0 [B, n], aref [B, m], D [B, m].  Returns (a_K, steps taken [B]).
    ``trace`` (a list) receives each step's (A_k, A'_k, taken) as bool tensors."""
    B, m, n = J.shape
    trM = torch.diagonal(M, dim1=-2, dim2=-1).sum(-1).detach()
    JT = J.mT.contiguous()
    a = a0
    done = torch.zeros(B, dtype=torch.bool, device=a0.device)
    steps = torch.zeros(B, dtype=torch.int32, device=a0.device)
    prev_act = None
    step_inf = None
    for k in range(K):
        d = a - a0
        r = (J @ a.unsqueeze(-1)).squeeze(-1) - aref
        act = r < 0
        Md = (M @ d.unsqueeze(-1)).squeeze(-1)
        F = Md + (JT @ (D * act * r).unsqueeze(-1)).squeeze(-1)
        with torch.no_grad():   # stop rule, evaluated at a_k
            conv = torch.linalg.vector_norm(F, dim=-1) <= tol * trM
            if k > 0:
                same = (act == prev_act).all(-1)
                conv = conv | (same & (step_inf <= tol * (1 + a.abs().amax(-1))))
            done = done | conv
        if bool(done.all()):
            break
        H = M + JT @ ((D * act).unsqueeze(-1) * J)
        p = -torch.linalg.solve(H, F)
        q = (J @ p.unsqueeze(-1)).squeeze(-1)
        Mp = (M @ p.unsqueeze(-1)).squeeze(-1)
        c0 = (p * Mp).sum(-1)
        b0 = (Mp * d).sum(-1)
        t, Ap = line_search(r.detach(), q.detach(), D.detach(), c0.detach(), b0.detach())
        w = D * Ap
        c = c0 + (w * q * q).sum(-1)
        b = b0 + (w * q * r).sum(-1)
        c = torch.where(done, torch.ones_like(c), c)    # no 0/0 on finished instances
        al = -b / c
        al = t + (al - al.detach())    # value of the search, derivative of -b/c
        step = al.unsqueeze(-1) * p
        a = torch.where(done.unsqueeze(-1), a, a + step)
        if trace is not None:
            trace.append((act.detach(), Ap.detach(), (~done).detach()))
        with torch.no_grad():
            step_inf = step.abs().amax(-1)
            steps += (~done).to(torch.int32)
        prev_act = act
    return a, steps


def vjp(M, J, a0, aref, D, abar, K: int, tol: float, trace=None):
    """Unrolled-AD gradient of abar . a_K with respect to (a0, aref, J, D, M).
    Returns dict(a, a0, aref, J, D, M, steps)."""
    leaves = [x.detach().requires_grad_(True) for x in (M, J, a0, aref, D)]
    with torch.enable_grad():
        aK, steps = solve(*leaves, K=K, tol=tol, trace=trace)
        gM, gJ, ga0, garef, gD = torch.autograd.grad((aK * abar).sum(), leaves, allow_unused=True)
    z = lambda g, x: torch.zeros_like(x) if g is None else g
    return dict(a=aK.detach(), a0=z(ga0, a0), aref=z(garef, aref), J=z(gJ, J), D=z(gD, D),
                M=z(gM, M), steps=steps)
