"""The packed-descriptor check every kernel runs before touching an instance
(cs_device.hpp, desc_ok), compiled for the host and run on the CPU.

Each case below violates exactly one condition (or sits exactly on a bound)
of: 1 <= n <= nmax, 0 <= m <= mmax, offsets >= 0, offset + extent <= total
for M (n^2), J (m n), the n-vectors (n) and the m-vectors (m).  Expected
values are written out by hand."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2607_24959_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# (n, m, onn, omn, on, om, nmax, mmax, tot_nn, tot_mn, tot_n, tot_m) -> expected
BIG = 2 ** 62
CASES = [
    ((3, 4, 0, 0, 0, 0, 3, 4, 9, 12, 3, 4), 1),          # one instance filling the batch
    ((3, 4, 7, 20, 5, 6, 3, 4, 16, 32, 8, 10), 1),       # every extent ends exactly at its total
    ((3, 4, 8, 20, 5, 6, 3, 4, 16, 32, 8, 10), 0),       # M one past the end
    ((3, 4, 7, 21, 5, 6, 3, 4, 16, 32, 8, 10), 0),       # J one past the end
    ((3, 4, 7, 20, 6, 6, 3, 4, 16, 32, 8, 10), 0),       # n-vectors one past the end
    ((3, 4, 7, 20, 5, 7, 3, 4, 16, 32, 8, 10), 0),       # m-vectors one past the end
    ((0, 4, 0, 0, 0, 0, 3, 4, 9, 12, 3, 4), 0),          # n = 0
    ((4, 4, 0, 0, 0, 0, 3, 4, 16, 16, 4, 4), 0),         # n above nmax (totals would fit)
    ((3, 5, 0, 0, 0, 0, 3, 4, 9, 15, 3, 5), 0),          # m above mmax (totals would fit)
    ((3, -1, 0, 0, 0, 0, 3, 4, 9, 12, 3, 4), 0),         # negative m
    ((3, 0, 0, 0, 0, 4, 3, 4, 9, 12, 3, 4), 1),          # no rows, m-offset at the end
    ((3, 4, -1, 0, 0, 0, 3, 4, 9, 12, 3, 4), 0),         # negative offset (M)
    ((3, 4, 0, -3, 0, 0, 3, 4, 9, 12, 3, 4), 0),         # negative offset (J)
    ((3, 4, 0, 0, -1, 0, 3, 4, 9, 12, 3, 4), 0),         # negative offset (n-vectors)
    ((3, 4, 0, 0, 0, -1, 3, 4, 9, 12, 3, 4), 0),         # negative offset (m-vectors)
    ((3, 4, BIG, 0, 0, 0, 3, 4, BIG + 8, 12, 3, 4), 0),  # near the int64 range: no overflow
    ((3, 4, BIG, 0, 0, 0, 3, 4, BIG + 9, 12, 3, 4), 1),
]

DRIVER = r"""
#include "cs_device.hpp"
#include <cstdio>
int main() {
    long long v[12];
    while (scanf("%lld %lld %lld %lld %lld %lld %lld %lld %lld %lld %lld %lld", &v[0], &v[1],
                 &v[2], &v[3], &v[4], &v[5], &v[6], &v[7], &v[8], &v[9], &v[10], &v[11]) == 12)
        printf("%d\n", (int)cs::desc_ok((int)v[0], (int)v[1], v[2], v[3], v[4], v[5], (int)v[6],
                                        (int)v[7], v[8], v[9], v[10], v[11]));
    return 0;
}
"""


def test_descriptor_check_cases():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "desc.hip")
        exe = os.path.join(d, "desc")
        open(src, "w").write(DRIVER)
        subprocess.check_call([HIPCC, "--cuda-host-only", "-std=c++17", f"-I{CSRC}", src, "-o", exe])
        inp = "".join(" ".join(str(x) for x in c) + "\n" for c, _ in CASES)
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    got = [int(x) for x in out.split()]
    assert got == [e for _, e in CASES], list(zip(got, [e for _, e in CASES]))
