"""GPU tests of the adaptive, non-nested symplectic Euler (Sec. 7) against the oracle.

- FP64 per-sample results equal the oracle's within 1e-12 on levels 0 to 4 (the merged
  time grid, the draw mapping and the coarse sign factors all agree), including the
  release at the ground and dt_0 = T/8, which only the adaptive rule makes stable;
- FP32 paths (step rule in FP32) agree with FP64 to rounding on level 0 and in law on
  coupled levels, where a tick of difference can re-pair the draws of a sample;
- the FP64 adaptive estimate takes the oracle driver's decisions;
- with the reference height at the cut-off the kernel reproduces uniform SE;
- several samples per wave (the per-wave hand-out), the 64-bit tick kernel, homogeneous
  turbulence (runs the uniform kernel) and the binned concentration path all match the
  oracle.
"""
import sys

import numpy as np
import pytest
from scipy.stats import ks_2samp

import oracle
import paper_1612_07717_amd as ld
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b, floor=1.0):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


@pytest.mark.parametrize("level,n", [(0, 2048), (1, 1999), (2, 1500), (4, 777)])
def test_fp64_samples_match_oracle(level, n):
    cfg = W.problem(integrator="SE", M0=40, x_adapt=50.0)
    say(f"adaptive SE level {level} n={n}")
    got = ld.level_samples(cfg, level, 3, n, "fp64")
    ref = oracle.level_samples(cfg, level, 3, n)
    err = _rel(got, ref)
    assert err.max() <= 1e-12, (err.max(), np.argmax(err) // 2)


def test_dt0_T_over_8_is_stable_and_matches_oracle():
    cfg = W.neutral(20.0, "SE", M0=8, x_adapt=50.0)      # uniform SE refuses this (6.45 > 2)
    got = ld.level_samples(cfg, 2, 0, 1024, "fp64")
    ref = oracle.level_samples(cfg, 2, 0, 1024)
    assert np.all(np.isfinite(got))
    assert _rel(got, ref).max() <= 1e-12


def test_fp32_paths_follow_the_fp64_law():
    """FP32 paths take their step rule in FP32, so their step ends can lie a tick away from
    the FP64 path's. One path alone (level 0) barely notices. A coupled sample does when
    such a tick makes or removes a coincidence of a fine and a coarse time point: the
    merged grid gains or loses an interval and every later xi_j moves to another interval,
    which makes the sample a fresh draw of the same scheme. So: level 0 agrees to rounding,
    and on level 2 most samples agree while the laws and the paired means agree."""
    cfg = W.problem(integrator="SE", M0=40, x_adapt=50.0)
    n = 8192
    a = ld.level_samples(cfg, 0, 0, n, "fp32")[:, 0]
    b = ld.level_samples(cfg, 0, 0, n, "fp64")[:, 0]
    d0 = np.abs(a - b)
    say(f"adaptive FP32 vs FP64 level 0: median {np.median(d0):.2e} m, 99% {np.quantile(d0, 0.99):.2e} m")
    assert np.median(d0) < 1e-3 and np.quantile(d0, 0.99) < 0.1
    a = ld.level_samples(cfg, 2, 0, n, "fp32")
    b = ld.level_samples(cfg, 2, 0, n, "fp64")
    d = np.abs(a - b)
    say(f"adaptive FP32 vs FP64 level 2: median {np.median(d):.2e} m, share within 1 cm {np.mean(d < 1e-2):.3f}")
    assert np.median(d) < 1e-2
    for col in range(2):
        assert ks_2samp(a[:, col], b[:, col]).pvalue > 1e-3
        diff = a[:, col] - b[:, col]
        assert abs(diff.mean()) <= 4.0 * diff.std() / np.sqrt(n) + 1e-3, (col, diff.mean())


def test_fp64_adaptive_estimate_matches_oracle_driver():
    cfg = W.problem(integrator="SE", M0=40, x_adapt=50.0)
    g = ld.estimate(2.0, cfg, precision="fp64", N_init=2000, L_max=7)
    o = oracle.estimate(2.0, cfg, N_init=2000, L_max=7)
    say(f"adaptive estimate N={g['N']} {g['estimate']:.6f} vs oracle N={o['N']} {o['estimate']:.6f}")
    assert g["N"] == o["N"] and g["L"] == o["L"]
    assert abs(g["estimate"] - o["estimate"]) <= 1e-11 * max(1.0, abs(o["estimate"]))


def test_reference_height_at_cutoff_is_uniform_se():
    cfg = W.problem(integrator="SE", M0=40)
    uni = ld.level_samples(cfg, 3, 0, 1024, "fp64")
    ada = ld.level_samples(dict(cfg, x_adapt=cfg["eps_reg"]), 3, 0, 1024, "fp64")
    assert _rel(ada, uni).max() <= 1e-12


def test_several_samples_per_lane_match_oracle_and_sums():
    """Above 2048 blocks of 256 lanes each lane runs several samples back to back: sampled
    per-sample parity with the oracle across the range (first, last, lane boundaries, a
    ragged tail), and the level sums equal the sums of the dumped samples."""
    cfg = W.problem(integrator="SE", M0=40, x_adapt=50.0)
    n, begin = 700_001, 5
    say(f"adaptive SE level 1 n={n} (several samples per lane)")
    got = ld.level_samples(cfg, 1, begin, n, "fp64")
    rng = np.random.default_rng(3)
    idx = sorted(set([0, 1, 255, 256, 524_287, 524_288, n - 1] + list(rng.integers(0, n, 25))))
    for i in idx:
        ref = oracle.level_samples(cfg, 1, begin + int(i), 1)[0]
        assert _rel(got[i], ref).max() <= 1e-12, (i, got[i], ref)
    s = ld.level_sums(cfg, 1, begin, n, "fp64")
    y = got[:, 0] - got[:, 1]
    assert s["n"] == n
    assert abs(s["sum_y"] - y.sum()) <= 1e-9 * np.abs(y).sum()
    assert abs(s["sum_y2"] - (y * y).sum()) <= 1e-9 * (y * y).sum()


def test_homogeneous_turbulence_never_adapts():
    """lambda is constant in homogeneous turbulence: the adaptive scheme is the uniform one
    (the library runs it as such) and equals the oracle's adaptive scheme per sample."""
    cfg = W.homogeneous(x_adapt=50.0)
    for level in (0, 3):
        got = ld.level_samples(cfg, level, 0, 1000, "fp64")
        ref = oracle.level_samples(cfg, level, 0, 1000)
        assert _rel(got, ref).max() <= 1e-12


def test_level_with_64_bit_ticks_matches_oracle():
    """M_7 = 40 * 2^7 = 5120 steps: T in ticks (5120 * 2^20) needs 64-bit counters, the
    other adaptive kernel; FP64 samples equal the oracle's."""
    cfg = W.problem(integrator="SE", M0=40, x_adapt=50.0)
    say("adaptive SE level 7 n=96 (64-bit ticks)")
    got = ld.level_samples(cfg, 7, 17, 96, "fp64")
    ref = oracle.level_samples(cfg, 7, 17, 96)
    assert _rel(got, ref).max() <= 1e-12


def test_binned_concentration_with_adaptive_steps_matches_oracle():
    """The p.d.f. path (dump of the level kernel, then the bins kernel) with adaptive
    steps: per-bin FP64 sums equal the oracle's."""
    cfg = W.problem(integrator="SE", M0=40, x_adapt=50.0, r=4, delta=100.0)
    g = ld.pdf_level_sums(cfg, 2, 3, 1500, 0.0, 50.0, 20, precision="fp64")
    o = oracle.pdf_level_sums(cfg, 2, 3, 1500, 0.0, 50.0, 20)
    for i, (x, y) in enumerate(zip(g, o)):
        assert x["n"] == y["n"] and x["n_nonfinite"] == y["n_nonfinite"], i
        for key in ("sum_y", "sum_y2", "sum_pf", "sum_pf2"):
            assert abs(x[key] - y[key]) <= 1e-12 * max(abs(x[key]), abs(y[key])) + 1e-12, (i, key)
