"""Pins of the smoothing polynomials, the compensated sums and the MLMC driver.

- p_r (Eq. 35): endpoint values and the moment conditions, integrated numerically in
  50-digit arithmetic from the oracle's coefficients;
- Neumaier sums against exact rational sums (Python fractions);
- the driver: the variance constraint sum_l V_l / N_l <= eps^2 / 2 (Eq. 17 split of
  Sec. 6) holds at exit, and over independent seeds the estimate's RMSE against the
  exact answer of a homogeneous problem (folded-Gaussian closed form) is <= eps.
"""
import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

import workloads as W
from test_oracle_closed_forms import continuous_mean_var, fold_mean

mp.mp.dps = 40


@pytest.mark.parametrize("r", [1, 2, 3, 4, 5, 6, 7, 8])
def test_smoothing_polynomial_definition(orc, r):
    c = orc.smoothing_poly(r)
    assert len(c) == r + 2
    poly = lambda s: sum(mp.mpf(float(ck)) * s**k for k, ck in enumerate(c))
    assert abs(poly(mp.mpf(-1)) - 1) < 1e-13
    assert abs(poly(mp.mpf(1))) < 1e-13
    for j in range(r):
        got = mp.quad(lambda s: s**j * poly(s), [-1, 0, 1])
        want = mp.mpf((-1) ** j) / (j + 1)
        assert abs(got - want) < 1e-12, (r, j, got, want)


def test_smoothing_polynomial_is_half_minus_odd(orc):
    """By symmetry of the conditions about s = 0, p_r - 1/2 is odd."""
    for r in (2, 4, 6, 8):
        c = orc.smoothing_poly(r)
        assert c[0] == pytest.approx(0.5, abs=1e-15)
        assert np.all(np.abs(c[2::2]) < 1e-12)


def test_level_sums_are_compensated_sums_of_samples(orc):
    """The per-level sums equal the exact rational sums of the per-sample values."""
    p = W.neutral(200.0, "GL")
    n = 3000
    for level in (0, 2):
        s = orc.level_sums(p, level, 17, n)
        pf_pc = orc.level_samples(p, level, 17, n)
        y = pf_pc[:, 0] - pf_pc[:, 1]
        exact = [sum(map(Fraction, y)), sum(Fraction(v) * Fraction(v) for v in y),
                 sum(map(Fraction, pf_pc[:, 0])),
                 sum(Fraction(v) * Fraction(v) for v in pf_pc[:, 0])]
        got = [s["sum_y"], s["sum_y2"], s["sum_pf"], s["sum_pf2"]]
        # each y*y is rounded once before summing; allow that plus a few ulps
        for g, e, k in zip(got, exact, range(4)):
            bound = 4 * np.finfo(float).eps * float(abs(e)) + (n * 1.2e-16 * float(abs(e)) if k in (1, 3) else 0)
            assert abs(Fraction(g) - e) <= Fraction(bound), (level, k)
        assert s["n"] == n and s["n_nonfinite"] == 0


def test_level_sums_are_split_invariant(orc):
    """Samples are indexed by counter, so two batches equal one (up to rounding)."""
    p = W.neutral(500.0, "BAOAB")
    a = orc.level_sums(p, 1, 0, 5000)
    b1 = orc.level_sums(p, 1, 0, 2000)
    b2 = orc.level_sums(p, 1, 2000, 3000)
    for k in ("sum_y", "sum_y2", "sum_pf", "sum_pf2"):
        assert b1[k] + b2[k] == pytest.approx(a[k], rel=1e-14)


def test_level_sums_do_not_depend_on_the_thread_count(orc):
    """Fixed-order chunks: one thread and all threads give the same bits."""
    p = W.neutral(300.0, "GL")
    many = orc.num_threads()
    a = orc.level_sums(p, 2, 3, 4000)
    orc.set_num_threads(1)
    try:
        b = orc.level_sums(p, 2, 3, 4000)
    finally:
        orc.set_num_threads(many)
    assert a == b


def test_plan_first_batch_and_variance_rule(orc):
    """N_l = ceil(2 eps^-2 sqrt(V_l/C_l) sum_k sqrt(V_k C_k)) after a first batch."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        L = int(rng.integers(1, 6))
        n = [int(rng.integers(100, 10000)) for _ in range(L + 1)]
        V = [float(10.0 ** rng.uniform(-4, 2)) * 4.0**-l for l in range(L + 1)]
        mean = [float(rng.normal(0, 1)) * 2.0**-l for l in range(L + 1)]
        s1 = [m * k for m, k in zip(mean, n)]
        s2 = [(v * (k - 1) + k * m * m) for v, k, m in zip(V, n, mean)]
        eps = float(10.0 ** rng.uniform(-3, -1))
        out = orc.plan(dict(L=L, n=n, sum1=s1, sum2=s2, M0=8, eps=eps, L_max=10, N_init=1000))
        C = [8 * 2**l for l in range(L + 1)]
        tot = sum(math.sqrt(v * c) for v, c in zip(out["V"], C))
        want = [max(0, math.ceil(2 * tot * math.sqrt(v / c) / eps**2) - k)
                for v, c, k in zip(out["V"], C, n)]
        if out["status"] == 0 and out["L"] == L:
            assert out["dn"] == want
        # the planned sample counts satisfy the variance constraint
        Nt = [k + d for k, d in zip(n, out["dn"])]
        if out["L"] == L:
            assert sum(v / m for v, m in zip(out["V"], Nt)) <= 0.5 * eps**2 * (1 + 1e-9)


def test_plan_adds_level_when_bias_too_large(orc):
    # level means halving (alpha = 1); bias estimate |Y_L| / (2 - 1) = 0.25 > eps/sqrt2
    L = 2
    n = [10**6] * 3
    mean = [10.0, 0.5, 0.25]
    V = [1e-8, 1e-8, 1e-8]
    s1 = [m * k for m, k in zip(mean, n)]
    s2 = [v * (k - 1) + k * m * m for v, k, m in zip(V, n, mean)]
    out = orc.plan(dict(L=L, n=n, sum1=s1, sum2=s2, M0=8, eps=0.1, L_max=10, N_init=1000, alpha=0))
    assert out["status"] == 0 and out["L"] == 3 and out["dn"][3] >= 1000
    assert out["alpha"] == pytest.approx(1.0) and out["bias_est"] == pytest.approx(0.25)
    # a given weak order is used as is: alpha = 2 -> bias max(0.25, 0.5/4) / 3
    out = orc.plan(dict(L=L, n=n, sum1=s1, sum2=s2, M0=8, eps=0.1, L_max=10, N_init=1000, alpha=2.0))
    assert out["alpha"] == 2.0 and out["bias_est"] == pytest.approx(0.25 / 3)
    # same, but converged bias
    out = orc.plan(dict(L=L, n=n, sum1=s1, sum2=s2, M0=8, eps=1.0, L_max=10, N_init=1000))
    assert out["status"] == 1
    # at L_max: stop, not converged
    out = orc.plan(dict(L=L, n=n, sum1=s1, sum2=s2, M0=8, eps=0.1, L_max=2, N_init=1000))
    assert out["status"] == 2


@pytest.mark.slow
@pytest.mark.parametrize("integ", ["SE", "BAOAB"])
def test_driver_rmse_within_eps(orc, integ):
    """Homogeneous turbulence released at 100 m with w0 = 0: the exact answer is the
    folded-Gaussian mean of the continuous integrated OU process."""
    mu, var = continuous_mean_var(1.3, 100.0, 1000.0, 100.0, 0.0)
    exact = fold_mean(mu, math.sqrt(var))
    eps = 4.0
    errs = []
    for seed in range(100, 140):
        p = W.homogeneous(integrator=integ, z0=100.0, release="fixed", w0=0.0, seed=seed)
        r = orc.estimate(eps, p, L_min=2, L_max=10, N_init=2000)
        assert r["status"] == 1 and r["n_nonfinite"] == 0
        Nl = r["N"]
        assert sum(v / n for v, n in zip(r["V"], Nl)) <= 0.5 * eps**2 * 1.02
        errs.append(r["estimate"] - exact)
    rmse = math.sqrt(np.mean(np.square(errs)))
    assert rmse <= eps, (rmse, errs)
