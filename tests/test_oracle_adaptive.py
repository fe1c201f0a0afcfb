"""Pins of the oracle's adaptive, non-nested symplectic Euler (Sec. 7).

- with the reference height at the cut-off (lambda(X_adapt) = lambda_max) no step adapts,
  and every coupled sample equals the uniform scheme's (Eqs. 8, 18, 31) to rounding;
- each path keeps its own law: the coarse path of level l and the fine path of level l-1
  follow the same adaptive rule, so their terminal laws agree (two-sample KS test);
- Var[Y_l] still decays like h_l^2 with the reflection sign factors (Sec. 7 and Sec. 4),
  and more slowly without them (the naive coupling);
- steps adapt only below the reference height: paths that stay above it follow the
  uniform scheme exactly;
- adaptivity reduces the mean level correction |E[Y_l]| of SE (the paper: a bias about
  6x smaller).
"""
import numpy as np
import pytest
from scipy.stats import ks_2samp

import workloads as W


def _se(**kw):
    return W.problem(integrator="SE", M0=40, **kw)


@pytest.mark.parametrize("level", [0, 1, 3])
def test_reference_height_at_cutoff_is_the_uniform_scheme(orc, level):
    cfg = _se()
    uni = orc.level_samples(cfg, level, 5, 1500)
    ada = orc.level_samples(dict(cfg, x_adapt=cfg["eps_reg"]), level, 5, 1500)
    scale = np.maximum(np.abs(uni), 1.0)
    assert np.max(np.abs(ada - uni) / scale) <= 1e-12


def test_coarse_path_has_the_previous_levels_fine_law(orc):
    cfg = _se(x_adapt=50.0)
    n = 6000
    coarse = orc.level_states(cfg, 3, 0, n)[:, 2]
    fine_prev = orc.level_states(dict(cfg, seed=4242), 2, 0, n)[:, 0]
    assert ks_2samp(coarse, fine_prev).pvalue > 1e-3
    # and it is not the law of the level's own fine path at a coarser resolution by accident:
    fine_same = orc.level_states(cfg, 3, 0, n)[:, 0]
    assert np.mean(np.abs(fine_same - coarse)) < 0.1 * np.std(coarse)


def _level_var(orc, cfg, level, n):
    s = orc.level_sums(cfg, level, 0, n)
    m = s["sum_y"] / s["n"]
    return s["sum_y2"] / s["n"] - m * m


@pytest.mark.slow
def test_variance_decays_like_h_squared_with_sign_factors(orc):
    cfg = _se(x_adapt=50.0)
    V = [_level_var(orc, cfg, l, 4000) for l in (2, 3, 4, 5)]
    ratios = np.array(V[:-1]) / np.array(V[1:])
    assert np.all(ratios > 2.5), ratios              # ~4 for beta = 2
    naive = dict(cfg, coupling="naive")
    Vn = [_level_var(orc, naive, l, 4000) for l in (3, 5)]
    assert Vn[1] > 2.0 * V[3], (Vn, V)                # without S: far larger at fine levels


def test_paths_above_the_reference_height_do_not_adapt(orc):
    """lambda decreases with height, so above X_adapt the ratio exceeds 1 and h_n = h: a
    release at 800 m followed for 100 s never comes near 50 m and is the uniform scheme."""
    cfg = _se(z0=800.0, T=100.0, x_adapt=50.0)
    for level in (0, 2):
        ada = orc.level_samples(cfg, level, 0, 1000)
        uni = orc.level_samples(dict(cfg, x_adapt=0.0), level, 0, 1000)
        assert np.max(np.abs(ada - uni) / np.maximum(np.abs(uni), 1.0)) <= 1e-12


def test_adaptivity_reduces_the_level_correction(orc):
    n = 20000
    uni = orc.level_sums(_se(), 2, 0, n)
    ada = orc.level_sums(_se(x_adapt=50.0), 2, 0, n)
    yu, ya = uni["sum_y"] / n, ada["sum_y"] / n
    se_a = np.sqrt(max(ada["sum_y2"] / n - ya * ya, 0.0) / n)
    assert abs(ya) + 3 * se_a < 0.5 * abs(yu), (ya, yu, se_a)
