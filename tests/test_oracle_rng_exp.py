"""Pins of the oracle's Philox4x32-10 and exp2s against things other than itself.

* Philox: bit-for-bit against rocRAND's host-callable engine (a library routine of the
  same published generator), compiled here from the installed header; plus
  uniformity of u = (r >> 8) 2^-24.
* exp2s: exact at integer arguments, relative error against float64 2^y within the
  bound of a degree-6 Taylor polynomial on [-1/2, 1/2] plus float rounding.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

ROCRAND_HDR = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref():
    if not os.path.exists(ROCRAND_HDR) or shutil.which("g++") is None:
        pytest.skip("rocRAND header or g++ not available")
    d = tempfile.mkdtemp(prefix="philox_ref_")
    exe = os.path.join(d, "philox_ref")
    subprocess.run(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(HERE, "philox_ref.cpp"), "-o", exe], check=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(123)
    rows = [[0, 0, 0, 0, 0, 0], [1, 0, 0, 0, 0, 0], [0, 1, 0, 0, 0, 0], [0, 0, 1, 0, 0, 0],
            [0, 0, 0, 1, 0, 0], [0, 0, 0, 0, 1, 0], [0, 0, 0, 0, 0, 1],
            [0xFFFFFFFF, 0, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF]]
    for _ in range(300):
        c = rng.integers(0, 2**32, size=6, dtype=np.uint64)
        c[1] %= 2**29  # the library derives this word from a 64-bit offset
        rows.append([int(v) for v in c])
    inp = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for r, line in zip(rows, out):
        want = [int(v) for v in line.split()]
        got = orc.philox4x32_10(r[:4], r[4:]).tolist()
        assert got == want, (r, got, want)


def test_uniform_conversion_exact(orc):
    assert orc.uniform(0) == 0.0
    assert orc.uniform(255) == 0.0
    assert orc.uniform(256) == 2.0 ** -24
    assert orc.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert orc.uniform(0x80000000) == 0.5


def test_philox_uniformity(orc):
    n = 20000
    us = np.empty(4 * n)
    for i in range(n):
        w = orc.philox4x32_10([i, 7, 3, 0], [0xDEADBEEF, 42])
        us[4 * i:4 * i + 4] = [orc.uniform(int(v)) for v in w]
    counts, _ = np.histogram(us, bins=64, range=(0.0, 1.0))
    assert stats.chisquare(counts).pvalue > 1e-4
    # adjacent counters are not correlated
    assert abs(np.corrcoef(us[:-4], us[4:])[0, 1]) < 0.02


def test_exp2s_integer_points_exact(orc):
    for n in range(-125, 40):
        assert orc.exp2s(float(n)) == 2.0 ** n


def test_exp2s_underflow_cut(orc):
    assert orc.exp2s(-125.0) == 2.0 ** -125
    assert orc.exp2s(-125.0001) == 0.0
    assert orc.exp2s(-1000.0) == 0.0


def test_exp2s_relative_error_bound(orc):
    # truncation (ln2/2)^7/7! ~ 1.2e-7 plus a few float roundings
    bound = 4e-7
    ys = np.concatenate([np.linspace(-125.0, 0.0, 40001), np.linspace(-0.5, 0.5, 2001),
                         np.linspace(0.0, 100.0, 2001)]).astype(np.float32)
    worst = 0.0
    for y in ys:
        v = orc.exp2s(float(y))
        ref = math.pow(2.0, float(y))
        worst = max(worst, abs(v - ref) / ref)
    assert worst < bound, worst


def test_exp2s_monotone_on_grid(orc):
    ys = np.linspace(-3.0, 3.0, 6001).astype(np.float32)
    vals = [orc.exp2s(float(y)) for y in ys]
    assert all(b >= a for a, b in zip(vals, vals[1:]))
