"""Other regularised constraint rows expressed with the solver's one-sided rows.

The solver's rows are one-sided: row i contributes 1/2 D_i min(r_i, 0)^2 with
r = J a - aref (the pyramid's edge rows, Sec. III-A).  Two further row kinds of
the reduced problem need no kernel of their own:

* a **limit** row (a joint or tendon limit) is one-sided already: it is a row
  of the same kind, with J the limit's Jacobian row and aref its reference
  acceleration;
* an **equality** row, whose cost is 1/2 D r^2 on both sides, is exactly two
  one-sided rows (J, aref) and (-J, -aref) with the same D:
  1/2 D min(r, 0)^2 + 1/2 D min(-r, 0)^2 = 1/2 D r^2, so the gradient is
  J^T D r and the Newton-matrix contribution D J^T J whichever side is active
  (at r = 0 exactly neither row is active: the one point where the reduced
  problem's second derivative has a jump of D J^T J).

`with_equality_rows` appends such pairs to a batch's rows; `fold_equality_grads`
maps the VJP of the expanded rows back to the equality rows.
"""
from __future__ import annotations

import torch


def with_equality_rows(J, aref, D, Je, arefe, De):
    """Append equality rows as one-sided pairs.  Shapes: J [B, m, n], aref and D
    [B, m] (m may be 0), Je [B, k, n], arefe and De [B, k].  Returns (J2, aref2,
    D2) with m + 2k rows: the original rows, then (Je, arefe), then (-Je, -arefe)."""
    J2 = torch.cat([J, Je, -Je], dim=-2).contiguous()
    aref2 = torch.cat([aref, arefe, -arefe], dim=-1).contiguous()
    D2 = torch.cat([D, De, De], dim=-1).contiguous()
    return J2, aref2, D2


def fold_equality_grads(Jbar, arefbar, Dbar, m, k):
    """VJP of the expanded rows -> (Jbar, arefbar, Dbar) of the original m rows and
    (Jebar, arefebar, Debar) of the k equality rows (the chain rule through the
    pair (Je, arefe, De), (-Je, -arefe, De))."""
    Jb = Jbar[..., :m, :], Jbar[..., m:m + k, :], Jbar[..., m + k:m + 2 * k, :]
    ab = arefbar[..., :m], arefbar[..., m:m + k], arefbar[..., m + k:m + 2 * k]
    Db = Dbar[..., :m], Dbar[..., m:m + k], Dbar[..., m + k:m + 2 * k]
    return (Jb[0], ab[0], Db[0]), (Jb[1] - Jb[2], ab[1] - ab[2], Db[1] + Db[2])
