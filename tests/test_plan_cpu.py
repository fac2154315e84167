"""CPU checks of the library's segmented line plans (no GPU needed).

* The closure rows the library builds (long-double column solves of the global
  A^-1 B) agree with the oracle's rows (transposed solves): two independent
  constructions of Eq. CS:fpCf.
* Replaying the GPU's per-line algorithm in NumPy from the library's own tables
  (wall rows, closure sums, Thomas runs) reproduces the oracle's sequential
  derivative, i.e. the plan tables are complete and consistent.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2203_00879_amd import nopcs

ALPHA, B1, B2 = 0.3793894912, 0.7877868952, 0.045801298


def line_plan(n, nseg, piece):
    lib = nopcs.lib()
    lib.nopcs_line_plan.argtypes = [ctypes.c_int32] * 4 + [ctypes.c_void_p] * 5
    nr, nc = ctypes.c_int32(), ctypes.c_int32()
    cap = 2 * n
    runs = np.zeros(2 * cap, np.int32)
    rows = np.zeros(cap, np.int32)
    coef = np.zeros(97 * cap)
    rc = lib.nopcs_line_plan(n, nseg, piece, cap, ctypes.byref(nr), runs.ctypes.data, ctypes.byref(nc),
                             rows.ctypes.data, coef.ctypes.data)
    assert rc == 0, nopcs.last_error()
    return runs[:2 * nr.value].reshape(-1, 2), rows[:nc.value], coef[:97 * nc.value].reshape(-1, 97)


def replay(f, runs, rows, coef, h=1.0):
    n = len(f)
    ih = 1.0 / h
    x = np.zeros(n)
    x[0] = 0.5 * ih * (4 * (f[1] - f[0]) - (f[2] - f[0]))
    x[1] = 0.5 * ih * (f[2] - f[0])
    x[n - 2] = 0.5 * ih * (f[n - 1] - f[n - 3])
    x[n - 1] = -0.5 * ih * (4 * (f[n - 2] - f[n - 1]) - (f[n - 3] - f[n - 1]))
    for q, e in enumerate(rows):
        j = np.arange(e - 48, e + 49)
        ok = (j >= 0) & (j < n)
        x[e] = ih * np.sum(coef[q][ok] * (f[j[ok]] - f[e]))
    d = np.zeros(n)
    for i in range(2, n - 2):
        d[i] = ih * (B1 * (f[i + 1] - f[i - 1]) + B2 * (f[i + 2] - f[i - 2]))
    known = np.zeros(n, bool)
    known[[0, 1, n - 2, n - 1]] = True
    known[rows] = True
    covered = known.copy()
    for lo, hi in runs:
        assert known[lo] and known[hi] and hi - lo >= 2
        m = hi - lo - 1
        assert not known[lo + 1:hi].any()
        covered[lo + 1:hi] = True
        cp = np.zeros(m + 1)
        dp = np.zeros(m + 1)
        for k in range(1, m + 1):
            i = lo + k
            r = d[i] - (ALPHA * x[lo] if k == 1 else 0) - (ALPHA * x[hi] if k == m else 0)
            den = 1.0 - (ALPHA * cp[k - 1] if k > 1 else 0.0)
            cp[k] = ALPHA / den
            dp[k] = (r - (ALPHA * dp[k - 1] if k > 1 else 0.0)) / den
        x[hi - 1] = dp[m]
        for k in range(m - 1, 0, -1):
            x[lo + k] = dp[k] - cp[k] * x[lo + k + 1]
    assert covered.all(), "plan leaves rows unsolved"
    return x


@pytest.mark.parametrize("n,nseg,piece", [(8, 1, 0), (32, 1, 0), (64, 4, 0), (100, 3, 12), (256, 8, 0),
                                          (256, 8, 16), (512, 4, -1), (130, 2, 17), (1024, 16, -1), (97, 24, 0)])
def test_plan_replay_matches_oracle(n, nseg, piece):
    runs, rows, coef = line_plan(n, nseg, piece)
    for q, e in enumerate(rows):
        ref = oracle.equiv_row(n, e)
        j = np.arange(e - 48, e + 49)
        ok = (j >= 0) & (j < n)
        # two independent constructions: agree to ~2 ulp of the row scale
        assert np.max(np.abs(coef[q][ok] - ref[j[ok]])) <= 4.5e-16 * max(1.0, np.max(np.abs(ref)))
        assert np.all(coef[q][~ok] == 0)
    rng = np.random.default_rng(n + nseg)
    f = rng.normal(size=n)
    got = replay(f, runs, rows, coef, h=1.0 / (n - 1))
    ref = oracle.d1_line(f, h=1.0 / (n - 1))
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_plan_rejects_bad_segmentation():
    lib = nopcs.lib()
    assert lib.nopcs_line_plan(16, 5, 0, 0, None, None, None, None, None) == nopcs.NOPCS_EINVAL
    assert lib.nopcs_line_plan(7, 1, 0, 0, None, None, None, None, None) == nopcs.NOPCS_EINVAL
