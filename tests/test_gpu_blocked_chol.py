"""The 256-thread blocked Cholesky and triangular solves.

Teams of 256 threads (the TEAM family for n > 32, the CHUNK family's n > 32
classes) factor the Newton matrix in 16-column blocks: the diagonal block in
registers, each panel row below it by a triangular solve against the block,
then the rank-16 trailing update.  The TEAM family keeps H at an odd row
stride (n | 1), so even n are padded and odd n are not.  These cases cover one
to seven blocks with full and ragged last blocks, at even and odd n, in FP64
against the oracle instance by instance (forward, IFT VJP and unrolled VJP,
whose tape stores the factor), and pivots that fail in the first and in a
later block (status ST_NOTSPD, outputs NaN).
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


SIZES = [33, 40, 47, 48, 64, 65, 96, 97]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("path", [N.PATH_TEAM, N.PATH_CHUNK])
def test_fp64_blocked_factor_sizes(n, path):
    _needs_gpu()
    if path == N.PATH_CHUNK and n > 96:
        # the CHUNK family pads n to a multiple of 16: FP64 n = 97 (112 padded)
        # does not fit its LDS plan, and the shape is refused
        with pytest.raises(N.CsError) as e:
            G.gpu_uniform(synth.uniform_batch(2, n, 8, 3400 + n), torch.float64, 60, 1e-12,
                          vjp=False, path=path)
        assert e.value.code == N.CS_EUNSUPPORTED
        return
    b = synth.uniform_batch(12, n, 8, 3400 + n)
    g = G.gpu_uniform(b, torch.float64, 60, 1e-12, path=path)
    o = G.oracle_uniform(b, 60, 1e-12)
    assert np.array_equal(g["status"], o["status"]), (n, path)
    conv = o["status"] == oracle.ST_CONVERGED
    assert conv.all(), (n, path)
    assert G.rel_rows(g["a"], o["a"], b.B).max() <= 1e-10, (n, path)
    assert np.array_equal(g["active"], o["active"]), (n, path)
    for k in G.GKEYS:
        e = G.rel_rows(g[k], o[k], b.B)
        assert e.max() <= 1e-9, (n, path, k, e.max())


@pytest.mark.parametrize("n", [36, 37])
@pytest.mark.parametrize("K", [1, 3, 10])
def test_fp64_unrolled_team_blocked(n, K):
    """The TEAM family's unrolled VJP records the factor of every step in its
    tape and reads it back in the reverse sweep (256 threads for n > 32).
    Iteration counts are compared exactly, so the tolerance is one where the
    oracle's counts do not move when it is scaled by 3 either way (at 1e-12 the
    gradient test sits at FP64 rounding for these n, and counts move by one)."""
    _needs_gpu()
    b = synth.uniform_batch(12, n, 8, 3500 + n)
    gu = G.gpu_unrolled_uniform(b, torch.float64, K, 1e-10, path=N.PATH_TEAM)
    ou = G.oracle_unrolled_uniform(b, K, 1e-10)
    assert np.array_equal(gu["status"], ou["status"]), (n, K)
    assert np.array_equal(gu["iters"], ou["iters"]), (n, K)
    assert G.rel_rows(gu["a"], ou["a"], b.B).max() <= 1e-10, (n, K)
    for k in G.GKEYS:
        e = G.rel_rows(gu[k], ou[k], b.B)
        assert e.max() <= 1e-8, (n, K, k, e.max())


@pytest.mark.parametrize("n", [40, 48])
@pytest.mark.parametrize("path", [N.PATH_TEAM, N.PATH_CHUNK])
def test_not_positive_definite_in_first_and_later_block(n, path):
    _needs_gpu()
    b = synth.uniform_batch(8, n, 4, 3600 + n)
    b.M[2] = -1e6 * np.eye(n)       # the first pivot fails
    b.M[5] = np.eye(n)
    b.M[5][n - 1, n - 1] = -1e6     # only the last pivot (third block) fails
    g = G.gpu_uniform(b, torch.float64, 60, 1e-12, vjp=False, path=path)
    for i in (2, 5):
        assert g["status"][i] == N.ST_NOTSPD and np.isnan(g["a"][i]).all(), (path, i)
    others = [i for i in range(8) if i not in (2, 5)]
    assert np.all(g["status"][others] == N.ST_CONVERGED), path
