"""The allocation-free level sums (mlmc_level_sums_noalloc) against mlmc_level_sums.

Both entry points run the same kernels on the same draws; the allocation-free one keeps
its block partials in the library's own device array instead of a caller workspace.
Through the C ABI, two calls in a row (the second on a smaller range, so the array
still holds the first call's partials beyond the second's) must each give exactly the
sums mlmc_level_sums gives, and in FP64 the sums must agree with the oracle's to
1e-12 of the sum of magnitudes (Sec. 3.3, Eq. 16).
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1612_07717_amd as ld
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(a, b):
    return a["s"] == b["s"] and a["c"] == b["c"] and a["n"] == b["n"] and \
        a["n_nonfinite"] == b["n_nonfinite"]


# (problem, precision, level, first sample, samples): STREAM and PIPE launches, large
# then smaller, so the second call of each pair reuses the array
CALLS = [
    (W.single_large("BAOAB"), "fp32", 2, 0, 300_000),     # STREAM, 1172 blocks
    (W.single_large("BAOAB"), "fp32", 8, 5, 5_000),       # PIPE (2048 steps), 79 blocks
    (W.neutral(300.0, "GL"), "fp64", 3, 0, 70_000),       # STREAM, 274 blocks
    (W.neutral(300.0, "SE"), "fp64", 2, 17, 1_001),       # STREAM, 4 blocks, ragged
]


@pytest.mark.parametrize("pair", [(0, 1), (2, 3), (1, 3)])
def test_noalloc_equals_level_sums_twice(pair):
    for k in pair:
        cfg, prec, level, begin, n = CALLS[k]
        say(f"case noalloc {cfg['integrator']} {prec} level={level} begin={begin} n={n}")
        got = ld.level_sums_noalloc(cfg, level, begin, n, prec)
        ref = ld.level_sums(cfg, level, begin, n, prec)
        assert got["n"] + got["n_nonfinite"] == n
        assert _same(got, ref), (got, ref)


def test_noalloc_fp64_matches_oracle():
    cfg = W.neutral(300.0, "BAOAB")
    level, begin, n = 3, 0, 3000
    say(f"case noalloc oracle BAOAB fp64 level={level} n={n}")
    got = ld.level_sums_noalloc(cfg, level, begin, n, "fp64")
    ref = oracle.level_sums(cfg, level, begin, n)
    assert got["n"] == ref["n"] == n and got["n_nonfinite"] == 0
    smp = oracle.level_samples(cfg, level, begin, n)
    y = smp[:, 0] - smp[:, 1]
    # each sample within 1e-12 relative of the oracle's -> sums within 1e-12 of sum |.|
    mag = {"sum_y": np.abs(y).sum(), "sum_y2": (y * y).sum(),
           "sum_pf": np.abs(smp[:, 0]).sum(), "sum_pf2": (smp[:, 0] ** 2).sum()}
    for k, m in mag.items():
        assert abs(got[k] - ref[k]) <= 1e-12 * m, (k, got[k], ref[k])


def test_noalloc_empty_range_writes_zero_sums():
    cfg = W.neutral(300.0, "GL")
    say("case noalloc empty range")
    got = ld.level_sums_noalloc(cfg, 4, 123, 0, "fp32")
    assert got["n"] == 0 and got["n_nonfinite"] == 0
    assert all(v == 0.0 for v in got["s"] + got["c"])
