"""GPU tests of the block modes and of the full-size workloads.

- A level range small enough for the wave-specialised (PIPE) blocks and the same range
  extended past that size (STREAM blocks) give bitwise identical per-sample results:
  both modes run the same arithmetic on the same draws, in the neutral layer and in
  homogeneous turbulence whose steps cross the whole layer.
- Full size: the single large estimate (neutral layer, BAOAB, dt_0 = T/8, levels
  0..12, relative eps 1e-4) in the launch configuration the benchmark times; sampled
  outputs are recomputed one by one by the oracle.
- The well-mixed test with 10^6 particles (uniform on [0, H] stays uniform) and the
  homogeneous closed forms at 10^6 samples per level.
"""
import math
import sys

import numpy as np
import pytest
from scipy import stats

import oracle
import paper_1612_07717_amd as ld
import workloads as W
from test_oracle_closed_forms import _level_law, fold_mean

pytestmark = pytest.mark.gpu

PIPE_MAX = 64 * 2048


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("integ,prec", [("BAOAB", "fp32"), ("GL", "fp64"), ("SE", "fp32"), ("BAOAB", "fp64")])
def test_pipe_and_stream_blocks_agree_bitwise(integ, prec):
    cfg = W.neutral(400.0, integ)          # M_0 = 40: level 3 has 320 fine steps
    say(f"case modes {integ} {prec}")
    pipe = ld.level_samples(cfg, 3, 11, PIPE_MAX, prec)        # PIPE blocks
    stream = ld.level_samples(cfg, 3, 11, PIPE_MAX + 1, prec)  # STREAM blocks
    assert np.array_equal(pipe, stream[:PIPE_MAX])
    s_pipe = ld.level_sums(cfg, 3, 11, 777, prec)
    ref = stream[:777]
    y = ref[:, 0] - ref[:, 1]
    assert s_pipe["n"] == 777
    assert abs(s_pipe["sum_y"] - y.sum()) <= 1e-12 * np.abs(y).sum()


def _lam_max(cfg):
    """lambda = sigma_U / (kappa_tau X_c) is largest at the lower cut-off (Eqs. 5, 7)."""
    e = cfg["eps_reg"]
    su = cfg["kappa_sigma"] * cfg["u_star"] * (1.0 - e / cfg["H"]) ** 0.75
    return su / (cfg["kappa_tau"] * e)


# Levels where a shorter expm1 series holds for the fine step h but not for the coarse
# step 2h (lambda_max h <= z < 2 lambda_max h): z = 1/16 (FP32) or 1/64 (FP64) between
# the full routine and the short series, z = 2^-8 (FP32) between the short series and
# the shortest. There the two paths of a sample take different expm1 code, in either
# block mode.
BOUNDARY = [("BAOAB", "fp32", 40, 5, 1 / 16), ("GL", "fp32", 40, 5, 1 / 16),
            ("BAOAB", "fp32", 8, 7, 1 / 16), ("GL", "fp32", 8, 7, 1 / 16),
            ("BAOAB", "fp64", 40, 7, 1 / 64), ("GL", "fp64", 40, 7, 1 / 64),
            ("BAOAB", "fp64", 8, 9, 1 / 64), ("GL", "fp64", 8, 9, 1 / 64),
            ("BAOAB", "fp32", 8, 11, 2.0 ** -8), ("GL", "fp32", 40, 9, 2.0 ** -8)]


@pytest.mark.parametrize("integ,prec,M0,level,z", BOUNDARY)
def test_pipe_and_stream_agree_on_the_short_series_boundary_level(integ, prec, M0, level, z):
    cfg = W.neutral(500.0, integ, M0=M0)
    h = cfg["T"] / (M0 << level)
    lam = _lam_max(cfg)
    assert lam * h <= z < 2.0 * lam * h
    say(f"case boundary {integ} {prec} M0={M0} level={level}")
    pipe = ld.level_samples(cfg, level, 3, PIPE_MAX, prec)        # PIPE blocks
    stream = ld.level_samples(cfg, level, 3, PIPE_MAX + 1, prec)  # STREAM blocks
    assert np.array_equal(pipe, stream[:PIPE_MAX])
    if prec == "fp64":
        ref = oracle.level_samples(cfg, level, 3, 48)
        tol = 1e-12 * np.maximum(np.abs(ref), 1e-3 * cfg["H"])
        assert np.all(np.abs(pipe[:48] - ref) <= tol)


# PIPE blocks advance their paths in chunks of 16 coarse steps (FP32 paths) or 8 (FP64);
# a path's last chunk is cut short where P = M_l / 2 is not a multiple of that. With
# M_0 = 41, level 3 has P = 164 (ragged in both precisions), level 4 P = 328 (FP32 only).
RAGGED = [("BAOAB", "fp32", 3), ("GL", "fp32", 3), ("SE", "fp32", 3), ("BAOAB", "fp32", 4),
          ("BAOAB", "fp64", 3), ("GL", "fp64", 3)]


@pytest.mark.parametrize("integ,prec,level", RAGGED)
def test_pipe_ragged_last_chunk_agrees_with_stream(integ, prec, level):
    cfg = W.neutral(500.0, integ, M0=41)
    P = (41 << level) // 2
    assert P % (16 if prec == "fp32" else 8) != 0
    say(f"case ragged {integ} {prec} level={level}")
    pipe = ld.level_samples(cfg, level, 7, PIPE_MAX, prec)        # PIPE blocks
    stream = ld.level_samples(cfg, level, 7, PIPE_MAX + 1, prec)  # STREAM blocks
    assert np.array_equal(pipe, stream[:PIPE_MAX])
    if prec == "fp64":
        ref = oracle.level_samples(cfg, level, 7, 48)
        tol = 1e-12 * np.maximum(np.abs(ref), 1e-3 * cfg["H"])
        assert np.all(np.abs(pipe[:48] - ref) <= tol)


@pytest.mark.parametrize("H", [100.0, 400.0])
@pytest.mark.parametrize("integ,prec", [("BAOAB", "fp32"), ("SE", "fp64"), ("GL", "fp64"), ("BAOAB", "fp64")])
def test_pipe_and_stream_agree_when_steps_cross_the_layer(integ, prec, H):
    """Homogeneous turbulence with sigma_w = 40 m/s and h = 3.125 s on level 3 (PIPE
    blocks, since M_3 = 320): with H = 100 m about 40 % of the steps are longer than the
    layer and fold by several reflections; with H = 400 m about a tenth of the samples
    have such a step (a plain OU simulation of the velocity gives 9.5 %). The two block
    modes agree bitwise, and FP64 paths match the oracle. A position's rounding error
    grows with the distance its path travels (about sigma_w T = 40 km here, some 10^2
    crossings of the layer) rather than with where it ends, so the scale below a
    position's magnitude is H itself instead of 10^-3 H."""
    cfg = W.homogeneous(H=H, sigma_u=40.0, z0=0.5 * H, M0=40, integrator=integ)
    say(f"case steps across the layer {integ} {prec} H={H}")
    pipe = ld.level_samples(cfg, 3, 5, PIPE_MAX, prec)
    stream = ld.level_samples(cfg, 3, 5, PIPE_MAX + 1, prec)
    diff = np.flatnonzero(np.any(pipe != stream[:PIPE_MAX], axis=1))
    assert diff.size == 0, (diff.size, diff[:8].tolist(), pipe[diff[:4]].tolist(), stream[diff[:4]].tolist())
    assert np.all((pipe >= 0.0) & (pipe <= H))
    if prec == "fp64":
        ref = oracle.level_samples(cfg, 3, 5, 700)
        err = np.abs(pipe[:700] - ref)
        say(f"  max |GPU - oracle| {err.max():.2e} m")
        assert np.all(err <= 1e-12 * np.maximum(np.abs(ref), H)), err.max()


def _sampled_parity(cfg, level, n, prec, k=48, seed=0):
    """Run the whole range on the GPU, recompute k sampled outputs with the oracle."""
    got = ld.level_samples(cfg, level, 0, n, prec)
    idx = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(seed).integers(0, n, k)]))
    ref = np.array([oracle.sample(cfg, level, int(i))[:2] for i in idx])
    return got[idx], ref


def test_full_size_sampled_parity_fp64():
    """The per-level sample counts of the large single estimate, FP64 paths: every
    sampled output within 1e-12 of the oracle's."""
    cfg = W.single_large("BAOAB")
    sizes = [(0, 19_713_142), (1, 574_618), (4, 25_751), (8, 10_000), (12, 10_000)]
    for level, n in sizes:
        say(f"case full-size fp64 level={level} n={n}")
        got, ref = _sampled_parity(cfg, level, n, "fp64", k=24 if level < 8 else 6)
        tol = 1e-12 * np.maximum(np.abs(ref), 1.0)
        assert np.all(np.abs(got - ref) <= tol), (level, np.abs(got - ref).max())


# FP32 paths against the oracle on the same draws: median and 90th percentile of the
# fine position's |error| (m) per level of the single large estimate, about 4x what the
# current kernels give (3.7e-5 / 1.0e-4 at level 0, 8.2e-5 / 2.4e-4 at level 3,
# 5.5e-4 / 1.4e-3 at level 8, 7.9e-3 / 1.6e-2 at level 12): FP32 rounding of a position
# near 500 m, accumulated over the path's half-steps.
FP32_ERROR_BOUNDS = {0: (1.5e-4, 4e-4), 3: (3.3e-4, 1e-3), 8: (2.2e-3, 5.5e-3), 12: (3.2e-2, 6.5e-2)}


def test_full_size_fp32_error_statement():
    """FP32 paths against the FP64 oracle on the same draws at the benchmark sizes:
    the per-sample position error stays at the FP32 rounding level in distribution."""
    cfg = W.single_large("BAOAB")
    for level, n, k in [(0, 19_713_142, 200), (3, 72_168, 200), (8, 10_000, 60), (12, 10_000, 40)]:
        say(f"case full-size fp32 level={level} n={n}")
        got, ref = _sampled_parity(cfg, level, n, "fp32", k=k)
        err = np.abs(got[:, 0] - ref[:, 0])
        med, q90 = np.median(err), np.quantile(err, 0.9)
        say(f"  fp32 fine |err| median {med:.3e} q90 {q90:.3e} max {err.max():.3e} m")
        bm, bq = FP32_ERROR_BOUNDS[level]
        assert med < bm and q90 < bq, (level, med, q90)
        if level > 0:
            errc = np.abs(got[:, 1] - ref[:, 1])
            assert np.median(errc) < bm and np.quantile(errc, 0.9) < bq, (level, np.median(errc))


def test_well_mixed_one_million_particles():
    """Sec. 2 well-mixed condition: 10^6 particles uniform on [0, H] with the conditional
    Gaussian velocity remain uniform at T (20 bins of 50 m), BAOAB, FP64 and FP32."""
    for prec in ("fp64", "fp32"):
        cfg = W.well_mixed("BAOAB", M0=160)
        x = ld.level_samples(cfg, 0, 0, 1_000_000, prec)[:, 0]
        counts, _ = np.histogram(x, bins=20, range=(0.0, 1000.0))
        chi2 = stats.chisquare(counts)
        say(f"well-mixed {prec}: chi2 {chi2.statistic:.1f} p {chi2.pvalue:.3g} "
            f"max dev {np.abs(counts / 50000 - 1).max():.4f}")
        assert chi2.pvalue > 1e-3


def _well_mixed_histogram(integ, M0, prec, n=1_000_000):
    x = ld.level_samples(W.well_mixed(integ, M0=M0), 0, 0, n, prec)[:, 0]
    counts, _ = np.histogram(x, bins=20, range=(0.0, 1000.0))
    return counts, stats.chisquare(counts)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_well_mixed_symplectic_euler_bias_shrinks_with_h(prec):
    """Sec. 2 and Sec. 3.1: symplectic Euler keeps the well-mixed law only up to its
    O(h) bias, which empties the lowest bin where lambda is large. With 10^6 particles
    the chi-square statistic and the lowest bin's deficit fall as h shrinks (M_0 = 40,
    160, 640; measured 3419, 150, 21.5 and -24 %, -4.5 %, -1.1 %), and at M_0 = 640 the
    histogram is uniform within its sampling error."""
    chi, low = [], []
    for M0 in (40, 160, 640):
        counts, c = _well_mixed_histogram("SE", M0, prec)
        say(f"well-mixed SE {prec} M0={M0}: chi2 {c.statistic:.1f} p {c.pvalue:.3g} "
            f"lowest bin {counts[0] / 50000 - 1:+.4f}")
        chi.append(c.statistic)
        low.append(abs(counts[0] / 50000 - 1))
    assert chi[0] > chi[1] > chi[2] and low[0] > low[1] > low[2]
    assert stats.chi2.sf(chi[2], 19) > 1e-3


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_well_mixed_geometric_langevin(prec):
    """The geometric Langevin scheme (Eq. 9) keeps the well-mixed law much better than
    symplectic Euler: its bias at M_0 = 40 (lowest bin +2 %) is visible with 10^6
    particles and gone at M_0 = 160, where the histogram is uniform (chi-square p >
    1e-3)."""
    counts40, c40 = _well_mixed_histogram("GL", 40, prec)
    counts160, c160 = _well_mixed_histogram("GL", 160, prec)
    say(f"well-mixed GL {prec}: chi2 {c40.statistic:.1f} (M0 40), {c160.statistic:.1f} (M0 160)")
    assert c40.statistic > c160.statistic
    assert c160.pvalue > 1e-3
    _, se40 = _well_mixed_histogram("SE", 40, prec)
    assert c40.statistic < 0.1 * se40.statistic


@pytest.mark.parametrize("integ", ["SE", "GL", "BAOAB"])
def test_homogeneous_closed_form_at_scale(integ):
    """10^6 samples per level: mean of the fine and coarse positions against the exact
    folded-Gaussian means of the per-level laws (release at 100 m, w0 = 0)."""
    cfg = W.homogeneous(integrator=integ, release="fixed", z0=100.0, w0=0.0)
    n = 1_000_000
    for level in (0, 2, 4):
        s = ld.level_samples(cfg, level, 0, n, "fp64")
        for col, lev in ((0, level), (1, level - 1)):
            if lev < 0:
                continue
            m, Cv = _level_law(cfg, integ, lev)
            exact = fold_mean(m[1], math.sqrt(Cv[1, 1]))
            x = s[:, col]
            assert abs(x.mean() - exact) < 4.5 * x.std() / math.sqrt(n), (level, lev, x.mean(), exact)
