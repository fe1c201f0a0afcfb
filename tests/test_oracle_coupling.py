"""Pins of the level coupling and the model's statistics in the neutral boundary layer.

- telescoping identity (Eq. 14): the coarse path of a level-l pair has the law of the
  fine path of level l-1, so the two are compared as independent samples;
- quadratic variance decay Var[Y_l] ~ h_l^2 with the reflection sign factors
  (Eqs. 31-32, Sec. 4) and the much slower decay of the naive coupling S = 1
  ("not even linear", Sec. 4.1.1);
- the well-mixed invariant (Sec. 2): a uniform initial distribution with the
  conditional Gaussian velocity stays uniform, up to the integrator's bias.
"""
import math

import numpy as np
import pytest
from scipy import stats

import workloads as W


@pytest.mark.parametrize("integ", ["SE", "GL", "BAOAB"])
def test_telescoping_coarse_path_has_previous_level_law(orc, integ):
    p = W.neutral(300.0, integ)
    n = 20000
    for level in (1, 2, 3):
        coarse = orc.level_states(p, level, 0, n)[:, 2]
        prev = orc.level_states(p, level - 1, 0, n)[:, 0]
        assert stats.ks_2samp(coarse, prev).pvalue > 1e-4
        se = math.sqrt(coarse.var() / n + prev.var() / n)
        assert abs(coarse.mean() - prev.mean()) < 4.5 * se


def _level_variances(orc, p, levels, n):
    V = []
    for l in levels:
        s = orc.level_sums(p, l, 0, n)
        m = s["sum_y"] / s["n"]
        V.append((s["sum_y2"] - s["n"] * m * m) / (s["n"] - 1))
    return np.array(V)


@pytest.mark.parametrize("integ", ["SE", "GL", "BAOAB"])
def test_variance_decays_quadratically_with_sign_factors(orc, integ):
    p = W.problem(integrator=integ)                 # Sec. 6.1 set-up, M_0 = 40
    V = _level_variances(orc, p, range(1, 6), 20000)
    rates = np.log2(V[:-1] / V[1:])
    assert rates.mean() > 1.7 and rates.min() > 1.5, rates


@pytest.mark.parametrize("integ", ["GL", "BAOAB"])
def test_naive_coupling_decays_slower_than_linear(orc, integ):
    p = W.problem(integrator=integ, coupling="naive")
    V = _level_variances(orc, p, range(1, 6), 20000)
    rates = np.log2(V[:-1] / V[1:])
    assert rates[1:].mean() < 1.0, rates
    # and it leaves the level means unbiased (Sec. 4.1.1): same E[Y_l] as the correct one
    good = W.problem(integrator=integ)
    for l in (2, 4):
        a = orc.level_sums(p, l, 0, 20000)
        b = orc.level_sums(good, l, 0, 20000)
        # same random numbers, so P_f is identical; compare the coarse means
        assert a["sum_pf"] == b["sum_pf"]
        ya, yb = a["sum_y"] / a["n"], b["sum_y"] / b["n"]
        va = a["sum_y2"] / a["n"] - ya * ya
        assert abs(ya - yb) < 4.5 * math.sqrt(va / a["n"])


@pytest.mark.parametrize("integ", ["GL", "BAOAB"])
def test_well_mixed_uniform_stays_uniform(orc, integ):
    p = W.well_mixed(integ, M0=160)
    st = orc.level_states(p, 0, 0, 100000)
    counts, _ = np.histogram(st[:, 0], bins=20, range=(0.0, 1000.0))
    assert stats.chisquare(counts).pvalue > 1e-3
    # conditional velocity law: U / sigma_U(X) ~ N(0, 1)
    su = np.array([orc.profile(p, x)[0] for x in st[:2000, 0]])
    assert stats.kstest(st[:2000, 1] / su, "norm").pvalue > 1e-4


def test_well_mixed_se_bias_shrinks_with_h(orc):
    """SE violates the invariant at coarse h (its O(h) bias near the ground) and
    approaches it as h -> 0."""
    dev = []
    for M0 in (40, 160, 640):
        st = orc.level_states(W.well_mixed("SE", M0=M0), 0, 0, 100000)
        c, _ = np.histogram(st[:, 0], bins=20, range=(0.0, 1000.0))
        dev.append(stats.chisquare(c).statistic)
    assert dev[0] > dev[1] > dev[2]
    assert stats.chi2.sf(dev[2], 19) > 1e-3
