"""Pins of the oracle's binned-concentration (vector QoI) path, Sec. 6.4.

- one bin is the scalar box QoI of Eqs. (34)/(37): identical sums, sample by sample;
- the smoothed bins telescope: their sums add up to the box spanning all of them;
- raw bins tiling (0, H] put every finite sample in exactly one bin;
- the vector planner with one bin takes the scalar planner's decisions, and with
  several bins it follows the bin of largest variance (the rule of Sec. 6.4);
- standard Monte Carlo draws N = ceil(2 max_i Var[P_i] / eps^2) samples of the single
  fine path and averages them;
- in homogeneous turbulence the MLMC and StMC estimates of every bin agree with the
  exact law of the continuous model (integrated OU position folded into [0, H]).
"""
import math

import numpy as np
import pytest

import workloads as W

H = 1000.0


def _box(cfg, a, b):
    return dict(cfg, qoi="p_box", qa=a, qb=b)


@pytest.mark.parametrize("level,r", [(0, 0), (2, 0), (0, 4), (3, 4)])
def test_one_bin_is_the_scalar_box(orc, level, r):
    cfg = W.neutral(300.0, "GL", r=r, delta=100.0)
    a, w = 250.0, 50.0
    vec = orc.pdf_level_sums(cfg, level, 7, 3000, a, w, 1)[0]
    sc = orc.level_sums(_box(cfg, a, a + w), level, 7, 3000)
    assert vec["n"] == sc["n"] and vec["n_nonfinite"] == sc["n_nonfinite"]
    assert vec["s"] == sc["s"] and vec["c"] == sc["c"]


def test_bins_telescope_to_the_spanning_box(orc):
    cfg = W.neutral(400.0, "BAOAB", r=4, delta=100.0)
    bins = orc.pdf_level_sums(cfg, 2, 0, 4000, 100.0, 50.0, 12)
    span = orc.level_sums(_box(cfg, 100.0, 700.0), 2, 0, 4000)
    for key in ("sum_y", "sum_pf"):
        tot = sum(b[key] for b in bins)
        assert tot == pytest.approx(span[key], rel=1e-12, abs=1e-9)


def test_raw_bins_tiling_the_layer_hold_every_sample(orc):
    cfg = W.well_mixed("SE", r=0, M0=40)
    n = 5000
    bins = orc.pdf_level_sums(cfg, 0, 0, n, 0.0, 50.0, 20)
    assert all(b["n"] == n for b in bins)
    # a position exactly at 0 falls in no (a, b] box; at most a handful may do so
    total = sum(b["sum_pf"] for b in bins)
    assert n - 2 <= total <= n
    counts = np.array([b["sum_pf"] for b in bins])
    assert np.all(counts == np.round(counts))


def _random_sums(rng, L, k, n):
    s1 = np.zeros((L + 1, k))
    s2 = np.zeros((L + 1, k))
    for l in range(L + 1):
        for i in range(k):
            mean = rng.normal(0, 0.05) * 2.0 ** -l
            var = 10 ** rng.uniform(-5, -1) * 4.0 ** -l
            s1[l, i] = mean * n[l]
            s2[l, i] = var * (n[l] - 1) + n[l] * mean * mean
    return s1, s2


def test_vector_planner_with_one_bin_is_the_scalar_planner(orc):
    rng = np.random.default_rng(5)
    for _ in range(400):
        L = int(rng.integers(0, 7))
        n = [int(rng.integers(10, 100000)) for _ in range(L + 1)]
        s1, s2 = _random_sums(rng, L, 1, n)
        eps = float(10 ** rng.uniform(-4, -1))
        common = dict(L=L, n=n, M0=int(rng.choice([8, 40, 80])), eps=eps,
                      L_max=int(rng.integers(L, 10)), fixed_L=int(rng.choice([-1, -1, L])),
                      N_init=1000, alpha=float(rng.choice([1.0, 2.0])))
        v = orc.pdf_plan(dict(common, n_bins=1, sum1=s1.tolist(), sum2=s2.tolist()))
        s = orc.plan(dict(common, sum1=s1[:, 0].tolist(), sum2=s2[:, 0].tolist(),
                          eps_is_relative=0, fixed_N=0))
        assert (v["status"], v["L"], v["dn"]) == (s["status"], s["L"], s["dn"])
        assert v["estimate"][0] == pytest.approx(s["estimate"], rel=1e-14, abs=1e-300)
        assert v["bias_est"] == pytest.approx(s["bias_est"], rel=1e-14, abs=1e-300)
        assert np.allclose(v["V"], s["V"], rtol=1e-14, atol=0)


def test_vector_planner_follows_the_bin_of_largest_variance(orc):
    rng = np.random.default_rng(6)
    L, n = 3, [40000, 9000, 3000, 1000]
    s1, s2 = _random_sums(rng, L, 3, n)
    # bin 1: the largest variance and the largest mean on every level
    for l in range(L + 1):
        m = 0.2 * 2.0 ** -l
        v = 0.3 * 4.0 ** -l
        s1[l, 1] = m * n[l]
        s2[l, 1] = v * (n[l] - 1) + n[l] * m * m
    common = dict(L=L, n=n, M0=40, eps=2e-3, L_max=8, fixed_L=-1, N_init=1000, alpha=1.0)
    vec = orc.pdf_plan(dict(common, n_bins=3, sum1=s1.tolist(), sum2=s2.tolist()))
    one = orc.pdf_plan(dict(common, n_bins=1, sum1=s1[:, 1:2].tolist(), sum2=s2[:, 1:2].tolist()))
    assert (vec["status"], vec["L"], vec["dn"]) == (one["status"], one["L"], one["dn"])
    assert vec["V"] == one["V"]


def test_stmc_draws_the_variance_rule_and_averages_the_fine_path(orc):
    cfg = W.neutral(200.0, "BAOAB", r=4, delta=100.0)
    eps, L = 1e-2, 2
    res = orc.estimate_pdf(eps, cfg, 0.0, 100.0, 10, estimator=orc.STMC, fixed_L=L, N_init=500)
    N = res["N"][0]
    fine = dict(cfg, M0=cfg["M0"] << L)
    bins = orc.pdf_level_sums(fine, 0, 0, N, 0.0, 100.0, 10)
    means = [b["sum_pf"] / b["n"] for b in bins]
    assert res["estimate"] == pytest.approx(means, rel=1e-14, abs=1e-15)

    def maxvar(bs):
        return max((b["sum_pf2"] - b["sum_pf"] ** 2 / b["n"]) / (b["n"] - 1) for b in bs)

    # N follows the pilot of 500 samples; the final variance asks for at most 1 % more
    pilot = maxvar(orc.pdf_level_sums(fine, 0, 0, 500, 0.0, 100.0, 10))
    assert N == math.ceil(2 * pilot / eps**2)
    assert math.ceil(2 * maxvar(bins) / eps**2) <= 1.01 * N
    assert res["fine_steps"] == N * (cfg["M0"] << L)


def _exact_bins(cfg, a0, w, k, coef):
    """E[P_i(X_T)] under the continuous homogeneous model (stationary Gaussian start)."""
    from test_oracle_closed_forms import continuous_mean_var
    mu, var = continuous_mean_var(cfg["sigma_u"], cfg["tau"], cfg["T"], cfg["z0"])
    sd = math.sqrt(var)
    xs = np.linspace(0.0, H, 400001)
    kk = np.arange(-40, 41)[:, None]
    dens = np.sum(np.exp(-0.5 * ((2 * kk * H + xs - mu) / sd) ** 2)
                  + np.exp(-0.5 * ((2 * kk * H - xs - mu) / sd) ** 2), axis=0) / (sd * math.sqrt(2 * math.pi))

    def g(s):
        s = np.clip(s, -1.0, 1.0)
        v = np.zeros_like(s)
        for c in coef[::-1]:
            v = v * s + c
        return v

    out = []
    for i in range(k):
        a, b = a0 + i * w, a0 + (i + 1) * w
        p = g((xs - b) / cfg["delta"]) - g((xs - a) / cfg["delta"])
        out.append(np.trapezoid(p * dens, xs))
    return np.array(out)


@pytest.mark.slow
@pytest.mark.parametrize("estimator", ["mlmc", "stmc"])
def test_homogeneous_bins_match_the_continuous_law(orc, estimator):
    cfg = W.homogeneous(r=4, delta=100.0)
    coef = orc.smoothing_poly(4)
    exact = _exact_bins(cfg, 0.0, 100.0, 10, coef)
    eps = 4e-3
    if estimator == "mlmc":
        res = orc.estimate_pdf(eps, cfg, 0.0, 100.0, 10, L_min=2, L_max=9, N_init=2000)
        assert res["status"] == 1
    else:
        res = orc.estimate_pdf(eps, cfg, 0.0, 100.0, 10, estimator=orc.STMC, fixed_L=6, N_init=2000)
    err = np.abs(np.array(res["estimate"]) - exact)
    assert err.max() <= 3 * eps, (err, res["N"], res["L"])
    assert abs(np.sum(res["estimate"]) - np.sum(exact)) <= 3 * eps
