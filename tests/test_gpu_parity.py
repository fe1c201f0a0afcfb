"""GPU parity: the HIP path against the CPU FP64 oracle, through the C ABI.

FP64 paths: every sample's P_l and P_{l-1} within 1e-12 relative of the oracle's
(relative to max(|P|, scale), scale = 1e-3 H for positions, 1e-3 sigma for velocities,
1 for indicators), on identical Philox draws. Positions that land within a few ulps of
a branch point (0, H, the cut-off heights) may take the other branch on one side; such
samples are counted and must stay below 1e-6 of the samples.

FP32 paths (same draws, 23-bit uniforms): the error is reported and bounded in
distribution, and the level means agree with FP64 far inside the statistical error.
"""
import math
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


def _scale(cfg):
    if cfg["qoi"] == "mean_z":
        return 1e-3 * cfg["H"]
    if cfg["qoi"] in ("velocity", "velocity_sq"):
        return 1e-3
    return 1.0


def _assert_fp64_parity(cfg, level, begin, n):
    say(f"case fp64 {cfg['integrator']} {cfg['profile']} {cfg['release']} {cfg['qoi']} "
        f"level={level} begin={begin} n={n}")
    got = ld.level_samples(cfg, level, begin, n, "fp64")
    ref = oracle.level_samples(cfg, level, begin, n)
    tol = 1e-12 * np.maximum(np.abs(ref), _scale(cfg))
    bad = np.abs(got - ref) > tol
    n_bad = int(bad.any(axis=1).sum())
    assert n_bad <= int(1e-6 * n), (n_bad, np.argwhere(bad)[:5], got[bad.any(axis=1)][:3],
                                    ref[bad.any(axis=1)][:3])
    return got, ref


CASES = []
for integ in ("SE", "GL", "BAOAB"):
    CASES.append(W.neutral(300.0, integ))
    CASES.append(W.problem(integrator=integ))                       # paper release 50 m, 0.1 m/s
    CASES.append(W.homogeneous(integrator=integ))
    CASES.append(W.well_mixed(integ))
CASES.append(W.neutral(700.0, "GL", qoi="p_above", qa=450.0, r=4, delta=100.0))
CASES.append(W.neutral(120.0, "BAOAB", qoi="p_box", qa=105.5, qb=155.5, r=0))
CASES.append(W.neutral(120.0, "SE", qoi="p_box", qa=105.5, qb=155.5, r=8, delta=100.0))
CASES.append(W.homogeneous(integrator="BAOAB", qoi="velocity_sq"))
CASES.append(W.neutral(500.0, "GL", qoi="velocity"))


@pytest.mark.parametrize("cfg", CASES, ids=lambda c: f"{c['integrator']}-{c['profile']}-{c['release']}-{c['qoi']}")
def test_per_sample_fp64_parity(cfg):
    for level, n in ((0, 2500), (1, 1300), (3, 777)):
        _assert_fp64_parity(cfg, level, 0, n)


def test_counter_high_word_and_odd_m0():
    cfg = W.neutral(400.0, "BAOAB")
    _assert_fp64_parity(cfg, 2, (1 << 32) - 300, 600)             # crosses the low-word wrap
    _assert_fp64_parity(dict(cfg, M0=37), 0, 5, 300)             # odd M_0 on level 0
    _assert_fp64_parity(dict(cfg, M0=37), 2, 5, 300)
    _assert_fp64_parity(dict(cfg, seed=(1 << 63) + 12345, stream_id=(1 << 24) - 1), 1, 0, 300)


def test_level_sums_match_oracle_and_samples():
    for cfg in (W.neutral(300.0, "GL"), W.homogeneous(), W.problem(integrator="SE")):
        for level, n in ((0, 20000), (2, 5000)):
            say(f"case sums {cfg['integrator']} level={level} n={n}")
            g = ld.level_sums(cfg, level, 0, n, "fp64")
            o = oracle.level_sums(cfg, level, 0, n)
            assert g["n"] == o["n"] == n and g["n_nonfinite"] == 0
            samples = oracle.level_samples(cfg, level, 0, n)
            y = samples[:, 0] - samples[:, 1]
            for k in ("sum_y", "sum_y2", "sum_pf", "sum_pf2"):
                ref = o[k]
                # each sample within 1e-12 relative -> sums within 1e-12 of sum |.|
                mag = {"sum_y": np.abs(y).sum(), "sum_y2": (y * y).sum(),
                       "sum_pf": np.abs(samples[:, 0]).sum(),
                       "sum_pf2": (samples[:, 0] ** 2).sum()}[k]
                assert abs(g[k] - ref) <= 1e-12 * mag + 1e-300, (k, g[k], ref)


def test_deterministic_and_batch_equivalent():
    cfg = W.neutral(250.0, "BAOAB")
    a = ld.level_sums(cfg, 2, 100, 30000, "fp32")
    b = ld.level_sums(cfg, 2, 100, 30000, "fp32")
    assert a == b
    batch = ld.level_sums_batch(cfg, [(0, 0, 50000), (3, 7, 3000), (1, 0, 20000)], "fp64")
    singles = [ld.level_sums(cfg, l, s, n, "fp64") for l, s, n in ((0, 0, 50000), (3, 7, 3000), (1, 0, 20000))]
    assert batch == singles


def test_empty_and_tiny_ranges():
    cfg = W.neutral(300.0, "GL")
    z = ld.level_sums(cfg, 1, 0, 0, "fp64")
    assert z["n"] == 0 and z["sum_y"] == 0.0 and z["sum_pf2"] == 0.0
    one = ld.level_sums(cfg, 1, 9, 1, "fp64")
    pf, pc, bad = oracle.sample(cfg, 1, 9)
    assert one["n"] == 1 and abs(one["sum_pf"] - pf) <= 1e-12 * max(abs(pf), 1.0)
    assert abs(one["sum_y"] - (pf - pc)) <= 1e-12 * max(abs(pf), 1.0)
    assert ld.level_samples(cfg, 2, 0, 0, "fp64").shape == (0, 2)


def test_split_invariance_on_device():
    cfg = W.neutral(300.0, "SE")
    whole = ld.level_sums(cfg, 2, 0, 40000, "fp64")
    parts = [ld.level_sums(cfg, 2, b, n, "fp64") for b, n in ((0, 12345), (12345, 27655))]
    for k in ("sum_y", "sum_y2", "sum_pf", "sum_pf2"):
        assert parts[0][k] + parts[1][k] == pytest.approx(whole[k], rel=1e-14)


def test_unstable_and_workspace_errors_on_device():
    with pytest.raises(ld.LdError) as e:
        ld.level_sums(W.single_large("SE"), 0, 0, 100)
    assert e.value.status == ld.LD_EUNSTABLE


@pytest.mark.parametrize("integ", ["SE", "GL", "BAOAB"])
def test_fp32_paths_against_fp64(integ):
    """FP32 paths on the same draws: per-sample error small in distribution, level
    means within a small fraction of the statistical error."""
    cfg = W.neutral(300.0, integ)
    n = 200000
    for level in (0, 3):
        say(f"case fp32 {integ} level={level}")
        s32 = ld.level_samples(cfg, level, 0, n, "fp32")
        s64 = ld.level_samples(cfg, level, 0, n, "fp64")
        dpf = np.abs(s32[:, 0] - s64[:, 0])
        assert np.quantile(dpf, 0.99) < 1e-3 * cfg["H"] * 1e-1     # 99% within 0.1 m
        assert np.median(dpf) < 1e-3
        y32, y64 = s32[:, 0] - s32[:, 1], s64[:, 0] - s64[:, 1]
        se = y64.std() / math.sqrt(n)
        assert abs(y32.mean() - y64.mean()) < 0.1 * se + 1e-6, (y32.mean(), y64.mean(), se)


def test_estimate_fixed_n_matches_oracle():
    """Homogeneous turbulence, levels 0..4, 10^4 samples per level, SE, FP64: the
    GPU estimate equals the oracle's to 1e-12 (same samples)."""
    cfg = W.homogeneous()
    g = ld.estimate(1.0, cfg, fixed_L=W.HOMOGENEOUS_LEVELS, fixed_N=True, N_init=W.HOMOGENEOUS_N)
    o = oracle.estimate(1.0, cfg, fixed_L=W.HOMOGENEOUS_LEVELS, fixed_N=True, N_init=W.HOMOGENEOUS_N)
    assert g["N"] == o["N"] == [W.HOMOGENEOUS_N] * (W.HOMOGENEOUS_LEVELS + 1)
    assert g["estimate"] == pytest.approx(o["estimate"], rel=1e-12)
    for a, b in zip(g["Yhat"], o["Yhat"]):
        assert abs(a - b) <= 1e-12 * 500.0
    # E[Z(T)] = 500 m exactly for a release at H/2 (symmetry of the folded law)
    assert abs(g["estimate"] - 500.0) < 4 * math.sqrt(g["stat_var"])


@pytest.mark.parametrize("integ", ["SE", "GL", "BAOAB"])
def test_adaptive_estimate_matches_oracle(integ):
    cfg = W.neutral(300.0, integ)
    g = ld.estimate(1e-2, cfg, eps_is_relative=True, L_max=9, N_init=5000)
    o = oracle.estimate(1e-2, cfg, eps_is_relative=True, L_max=9, N_init=5000)
    say(f"estimate {integ}: gpu {g['estimate']} N={g['N']} oracle {o['estimate']} N={o['N']}")
    assert g["N"] == o["N"] and g["L"] == o["L"] and g["status"] == o["status"] == 1
    assert g["estimate"] == pytest.approx(o["estimate"], rel=1e-11)
