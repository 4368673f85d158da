"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every function include/cs.h declares, answer
size queries with the documented layouts, and reject bad arguments before
anything reaches a GPU.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest
import torch

from paper_2607_24959_amd import _native as N
from paper_2607_24959_amd import solver

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"\b(cs_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    decl = _declared()
    assert set(decl) == set(N.EXPORTED)
    L = N.lib()
    for name in decl:
        assert hasattr(L, name), name


def test_version_and_strerror():
    assert N.version() == 1
    assert N.strerror(0) == "ok"
    assert "invalid" in N.strerror(-1)
    assert "small" in N.strerror(-2)


def test_state_and_tape_sizes_uniform():
    b = solver.Batch.uniform(4096, 9, 64, torch.float32, device="cpu")
    al = lambda x: (x + 255) // 256 * 256
    assert b.state_bytes() == al(4 * 4096 * 45) + 4096 * 64
    for K in (0, 1, 10):
        recT = 2 * 9 + 45 + 2 * 64 + 2
        assert b.tape_bytes(K) == al(4 * K * 4096 * recT) + K * 2 * 4096 * 64
    b64 = solver.Batch.uniform(64, 6, 16, torch.float64, device="cpu")
    assert b64.state_bytes() == al(8 * 64 * 21) + 64 * 16


def test_tape_grows_linearly_in_K():
    b = solver.Batch.uniform(1024, 18, 128, torch.float32, device="cpu")
    s = [b.tape_bytes(K) for K in range(1, 11)]
    d = np.diff(s)
    assert np.all(np.abs(d - d[0]) <= 256)


def test_state_and_tape_sizes_packed():
    nv = np.array([3, 9, 96, 18])
    nr = np.array([0, 64, 1024, 12])
    b = solver.Batch.packed_from(nv, nr, torch.float32, device="cpu")
    al = lambda x: (x + 255) // 256 * 256
    assert b.state_bytes() == al(4 * int((nv * (nv + 1) // 2).sum())) + int(nr.sum())
    K = 3
    recT = int((2 * nv + nv * (nv + 1) // 2 + 2 * nr + 2).sum())
    assert b.tape_bytes(K) == al(4 * K * recT) + K * 2 * int(nr.sum())


def _desc(**kw):
    d = N.CsBatch()
    d.B, d.dtype, d.nv_uniform, d.nrows_uniform = 4, N.CS_F32, 9, 64
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def _fwd(desc, params=None, state_nbytes=1 << 30, ptr=C.c_void_p(16)):
    p = params or N.CsSolverParams(10, 0, 1e-5)
    return N.forward(desc, p, ptr, ptr, ptr, ptr, ptr, None, ptr, ptr, state_nbytes, ptr, None, None)


def test_argument_validation_before_launch():
    assert _fwd(_desc(dtype=7)) == N.CS_EINVAL
    assert _fwd(_desc(nv_uniform=0)) == N.CS_EINVAL
    assert _fwd(_desc(nv_uniform=N.NV_MAX + 1)) == N.CS_EINVAL
    assert _fwd(_desc(nrows_uniform=-1)) == N.CS_EINVAL
    assert _fwd(_desc(B=-1)) == N.CS_EINVAL
    assert _fwd(_desc(), N.CsSolverParams(-1, 0, 1e-5)) == N.CS_EINVAL
    assert _fwd(_desc(), N.CsSolverParams(10, 1, 1e-5)) == N.CS_EINVAL
    assert _fwd(_desc(), N.CsSolverParams(10, 3, 1e-5)) == N.CS_EINVAL
    assert _fwd(_desc(), N.CsSolverParams(10, N.FORWARD_CG | 1, 1e-5)) == N.CS_EINVAL
    assert _fwd(_desc(dtype=7), N.CsSolverParams(10, N.FORWARD_CG, 1e-5)) == N.CS_EINVAL
    assert _fwd(_desc(), N.CsSolverParams(10, 0, float("nan"))) == N.CS_EINVAL
    assert _fwd(_desc(), N.CsSolverParams(10, 0, -1.0)) == N.CS_EINVAL
    assert _fwd(_desc(), state_nbytes=16) == N.CS_ENOSPC
    assert _fwd(_desc(), ptr=None) == N.CS_EINVAL
    # a packed descriptor missing one of its arrays
    assert _fwd(_desc(nv=16)) == N.CS_EINVAL
    # empty batch is a no-op
    assert _fwd(_desc(B=0)) == N.CS_OK


def test_unrolled_tape_too_small_is_enospc():
    d = _desc()
    p = N.CsSolverParams(5, 0, 1e-5)
    ptr = C.c_void_p(16)
    rc = N.unrolled_vjp(d, p, ptr, ptr, ptr, ptr, ptr, ptr, ptr, ptr, ptr, ptr, ptr, ptr, ptr,
                        N.tape_bytes(d, 5) - 1, ptr, None, None)
    assert rc == N.CS_ENOSPC


def test_vjp_state_too_small_is_enospc():
    d = _desc()
    ptr = C.c_void_p(16)
    rc = N.ift_vjp(d, ptr, N.state_bytes(d) - 1, ptr, ptr, ptr, ptr, ptr, ptr, ptr, ptr, ptr,
                   ptr, ptr, ptr, None)
    assert rc == N.CS_ENOSPC


def test_batch_wrapper_checks_shapes():
    b = solver.Batch.uniform(4, 3, 8, torch.float32, device="cpu")
    with pytest.raises(ValueError):
        b.check("J", torch.zeros(4, 8, 2), 4 * 8 * 3)
    with pytest.raises(ValueError):
        b.check("J", torch.zeros(4, 8, 3, dtype=torch.float64), 4 * 8 * 3)
    with pytest.raises(ValueError):
        solver.Batch.packed_from(np.array([3, 0]), np.array([4, 4]), device="cpu")


def test_static_tape_entry_rejects_before_any_launch():
    """cs_unrolled_vjp_static checks its limits on the host: a tape larger than
    the static array is CS_ENOSPC, a RECORD/REPLAY phase is CS_EINVAL."""
    b = solver.Batch.uniform(4096, 9, 64, torch.float32, device="cpu")
    big = 1
    while b.tape_bytes(big) <= N.STATIC_TAPE_BYTES:
        big += 1
    p = N.CsSolverParams(big, 0, 1e-5)
    z = C.c_void_p(16)   # never dereferenced: the call returns before any launch
    args = [z] * 12 + [z, z, None]
    assert N.unrolled_vjp_static(b.desc, p, *args) == N.CS_ENOSPC
    for flags in (1, 2):
        p = N.CsSolverParams(10, flags, 1e-5)
        assert N.unrolled_vjp_static(b.desc, p, *args) == N.CS_EINVAL


def test_rollout_workspace_and_argument_validation():
    """cs_rollout_workspace_bytes: per step, the factors (256-aligned) then the
    active sets (256-aligned), or the active sets alone when recomputing;
    invalid parameters give 0 bytes and CS_EINVAL before any launch."""
    b = solver.Batch.uniform(4, 6, 8, torch.float64, device="cpu")
    al = lambda x: (x + 255) // 256 * 256
    P = lambda T, flags, **kw: N.CsRolloutParams(T, flags, kw.get("max_iter", 20), kw.get("res", 0),
                                                 kw.get("tol", 1e-12), 0.002, 100.0)
    step = al(8 * 4 * 21) + al(4 * 8)
    assert N.rollout_workspace_bytes(b.desc, P(3, 3)) == 3 * step
    assert N.rollout_workspace_bytes(b.desc, P(3, 1)) == 3 * step
    assert N.rollout_workspace_bytes(b.desc, P(3, 7)) == 3 * al(4 * 8)
    for bad in (P(0, 3), P(3, 0), P(3, 8), P(3, 4), P(3, 3, max_iter=-1), P(3, 3, res=1),
                P(3, 3, tol=float("nan"))):
        assert N.rollout_workspace_bytes(b.desc, bad) == 0
        rc = N.rollout(b.desc, bad, *([None] * 11), None, 0, None, None, None)
        assert rc == N.CS_EINVAL
    # required pointers are checked before any launch
    ws = C.c_void_p(1)
    rc = N.rollout(b.desc, P(3, 1), None, None, None, None, None, None, None, None, None, None,
                   None, ws, 1 << 20, None, None, None)
    assert rc == N.CS_EINVAL


def test_round_cone_entry_points_validate_before_launch():
    """Rows not a multiple of 3 in a uniform batch, flags != 0 and missing
    pointers are CS_EINVAL; a short state buffer is CS_ENOSPC -- all before any
    launch."""
    b = solver.Batch.uniform(4, 6, 10, torch.float64, device="cpu")
    p = N.CsSolverParams(10, 0, 1e-10)
    one = C.c_void_p(1)
    assert N.forward_ell(b.desc, p, *([one] * 10), 1 << 20, one, None, None) == N.CS_EINVAL
    b3 = solver.Batch.uniform(4, 6, 12, torch.float64, device="cpu")
    assert N.forward_ell(b3.desc, N.CsSolverParams(10, 4, 1e-10), *([one] * 10), 1 << 20, one,
                         None, None) == N.CS_EINVAL
    assert N.forward_ell(b3.desc, p, None, *([one] * 9), 1 << 20, one, None, None) == N.CS_EINVAL
    assert N.forward_ell(b3.desc, p, *([one] * 10), 16, one, None, None) == N.CS_ENOSPC
    assert N.ift_vjp_ell(b.desc, one, 1 << 20, *([one] * 9), *([None] * 7), None) == N.CS_EINVAL


def test_mixed_rows_entry_points_validate_before_launch():
    b = solver.Batch.uniform(4, 6, 12, torch.float64, device="cpu")
    p = N.CsSolverParams(10, 0, 1e-10)
    one = C.c_void_p(1)
    assert N.forward_rows(b.desc, N.CsSolverParams(10, 4, 1e-10), *([one] * 10), 1 << 20, one,
                          None, None) == N.CS_EINVAL
    assert N.forward_rows(b.desc, p, None, *([one] * 9), 1 << 20, one, None, None) == N.CS_EINVAL
    assert N.forward_rows(b.desc, p, *([one] * 10), 16, one, None, None) == N.CS_ENOSPC
    assert N.ift_vjp_rows(b.desc, one, 1 << 20, None, *([one] * 8), *([None] * 6), None) == \
        N.CS_EINVAL
