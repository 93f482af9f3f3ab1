"""The term thresholds of the layer build (term_thresholds in csrc/ara_math.hpp,
compiled for the host from the library's own source) against scipy's
regularized incomplete beta.

A draw z of an entry with shapes (a, b) and maximum loss m has loss m x with
x = I^{-1}_z(a, b) (section 3.3), and an XELT term min(max(l - ret, 0), lim)
(section 2.3) that is 0 when x <= ret/m and lim when x >= (ret+lim)/m, i.e.
when z <= I_{ret/m} or z >= I_{(ret+lim)/m}.  The layer kernels skip the
inverse exactly for z <= thr_lo or z >= thr_hi, so these must hold:
thr_lo <= I_{ret/m} and thr_hi >= I_{(ret+lim)/m} (never skip a draw the
terms do not fix), each within one code step (1/255) plus the margin, and
the special cases: no retention never skips low, no limit never skips high,
a retention at or beyond m always skips, a degenerate entry skips by its mean.
"""
import os
import subprocess

import numpy as np
import pytest
from scipy.special import betainc

from conftest import ROOT

EMU = os.path.join(ROOT, "tests", "emu")
CXX = os.environ.get("EMU_CXX", "/opt/rocm/llvm/bin/clang++")

pytestmark = pytest.mark.skipif(not os.path.exists(CXX), reason="host clang++ not found")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("thr") / "thr_driver")
    subprocess.check_call([CXX, "-std=c++20", "-O1", "-Wno-unknown-attributes", "-Wno-ignored-attributes",
                           "-I", EMU, "-I", os.path.join(ROOT, "include"), "-o", exe,
                           os.path.join(EMU, "thr_driver.cpp"), os.path.join(EMU, "emu_runtime.cpp"), "-pthread"])
    return exe


def _run(driver, rows):
    inp = "\n".join(" ".join(repr(float(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([driver], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    vals = np.array([[float(x) for x in line.split()] for line in out if line.strip()])
    return vals[:, 0].astype(int), vals[:, 1].astype(int), vals[:, 2], vals[:, 3]


def test_thresholds_bound_the_exact_probabilities(driver):
    rng = np.random.default_rng(7)
    n = 4000
    a = np.exp(rng.uniform(np.log(3e-3), np.log(40.0), n))
    b = np.exp(rng.uniform(np.log(3e-3), np.log(40.0), n))
    m = np.exp(rng.uniform(np.log(1e4), np.log(1e7), n))
    ret = m * rng.uniform(0.0, 0.9, n)
    lim = m * rng.uniform(0.0, 0.9, n)
    cl, ch, lo, hi = _run(driver, np.stack([a, b, m, ret, lim], 1))
    m32 = m.astype(np.float32).astype(np.float64)            # the library keeps max_l in FP32
    il = betainc(a, b, np.minimum(ret / m32, 1.0))
    ih = betainc(a, b, np.minimum((ret + lim) / m32, 1.0))
    never_hi = (ret + lim) / m32 >= 1.0
    # never skips a draw whose term the quantile could change
    assert np.all(lo <= il)
    assert np.all(hi[~never_hi] >= ih[~never_hi])
    # and skips all but at most one code step (and the margin) of those it could
    step = 1.0 / 255.0 + 1e-6
    assert np.all(il - lo <= step)
    tight = ~never_hi & (ch < 255)
    assert np.all(hi[tight] - ih[tight] <= step)
    assert np.all(ch[never_hi] == 255)


def test_threshold_special_cases(driver):
    rows = [
        (2.0, 5.0, 1e6, 0.0, 3e5),        # no retention: never skip low
        (2.0, 5.0, 1e6, 1e5, np.inf),     # no limit: never skip high
        (2.0, 5.0, 1e6, 1e6, 1e5),        # retention at max_l: every draw nets to 0
        (2.0, 5.0, 1e6, 2e6, 1e5),        # beyond it
        (0.0, 0.0, 3e5, 4e5, 1e5),        # degenerate, mean 3e5 within the retention
        (0.0, 0.0, 3e5, 1e5, 1e5),        # degenerate, mean beyond retention + limit
        (0.0, 0.0, 3e5, 1e5, 5e5),        # degenerate, mean between
        (2.0, 5.0, 1e6, 2e5, 0.0),        # zero limit: one threshold, both sides skip
    ]
    cl, ch, lo, hi = _run(driver, rows)
    assert lo[0] == 0.0 and hi[1] >= 1.0
    assert lo[2] == 1.0 and lo[3] == 1.0
    assert lo[4] == 1.0
    assert lo[5] == 0.0 and hi[5] == 0.0
    assert lo[6] == 0.0 and hi[6] >= 1.0
    i = betainc(2.0, 5.0, 2e5 / float(np.float32(1e6)))
    assert lo[7] <= i <= hi[7] and hi[7] - lo[7] <= 2.0 / 255.0 + 1e-6
