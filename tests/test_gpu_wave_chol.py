"""The one-wave register Cholesky and triangular solves.

Every one-wave team (the TEAM and CHUNK families for n <= 32, the fused
rollout, the round cone, the mixed rows) factors the Newton matrix with lane
i holding row i in registers, 16 or 32 of them chosen by n.  These cases sit
on both sides of that bound (n = 15, 16, 17, 31, 32) and at n = 1, 2, in FP64
(forward and IFT VJP against the oracle, instance by instance: a within
1e-10, the status equal, the gradients of converged instances within 1e-9)
and for a not positive definite M (status ST_NOTSPD, outputs NaN); the
one-wave line search at row counts on both sides of its register bound.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2607_24959_amd import synth
from paper_2607_24959_amd import _native as N

import gpu_common as G

pytestmark = pytest.mark.gpu


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("n", [1, 2, 15, 16, 17, 31, 32])
@pytest.mark.parametrize("path", [N.PATH_TEAM, N.PATH_CHUNK])
def test_fp64_register_factor_sizes(n, path):
    _needs_gpu()
    b = synth.uniform_batch(48, n, 8, 3100 + n)
    g = G.gpu_uniform(b, torch.float64, 60, 1e-12, path=path)
    o = G.oracle_uniform(b, 60, 1e-12)
    assert np.array_equal(g["status"], o["status"]), (n, path)
    ea = G.rel_rows(g["a"], o["a"], b.B)
    assert ea.max() <= 1e-10, (n, path, ea.max())
    conv = o["status"] == oracle.ST_CONVERGED
    assert conv.all()
    for k in G.GKEYS:
        e = G.rel_rows(g[k], o[k], b.B)[conv]
        assert e.max() <= 1e-9, (n, path, k, e.max())


@pytest.mark.parametrize("n", [16, 17])
def test_not_positive_definite_on_either_side_of_the_bound(n):
    _needs_gpu()
    b = synth.uniform_batch(8, n, 4, 3200 + n)
    b.M[2] = -1e6 * np.eye(n)       # the first pivot fails
    b.M[5] = np.eye(n)
    b.M[5][n - 1, n - 1] = -1e6     # only the last pivot fails
    g = G.gpu_uniform(b, torch.float64, 60, 1e-12, vjp=False, path=N.PATH_TEAM)
    for i in (2, 5):
        assert g["status"][i] == N.ST_NOTSPD and np.isnan(g["a"][i]).all(), i
    others = [i for i in range(8) if i not in (2, 5)]
    assert np.all(g["status"][others] == N.ST_CONVERGED)


@pytest.mark.parametrize("nc", [15, 16, 17, 48, 64, 65])
def test_fp64_wave_line_search_row_counts(nc):
    """The one-wave line search keeps up to four rows per lane in registers
    (m <= 256) and falls back to the team form beyond: m = 60 .. 260 rows
    through the TEAM family (one wave for n <= 32), FP64 against the oracle."""
    _needs_gpu()
    b = synth.uniform_batch(32, 9, nc, 3300 + nc)
    g = G.gpu_uniform(b, torch.float64, 60, 1e-12, path=N.PATH_TEAM)
    o = G.oracle_uniform(b, 60, 1e-12)
    assert np.array_equal(g["status"], o["status"]), nc
    assert np.all(o["status"] == oracle.ST_CONVERGED)
    assert G.rel_rows(g["a"], o["a"], b.B).max() <= 1e-10, nc
    assert np.array_equal(g["active"], o["active"]), nc
    for k in G.GKEYS:
        e = G.rel_rows(g[k], o[k], b.B)
        assert e.max() <= 1e-9, (nc, k, e.max())
