"""Closed-form pins of the oracle in homogeneous turbulence.

With constant sigma_U and tau the drift dV/dX vanishes and the extended SDE of
Sec. 4 (Eqs. 21-23) is the free one, so each scheme's position is exactly the fold
of a Gaussian whose mean and covariance follow a 2x2 linear recursion. These tests

1. check that the recursion's law converges to the continuous-time law (textbook
   integrated OU process) at the weak orders the paper states (first order for SE
   and GL, Sec. 3.1; BAOAB second order when the profile is constant, App. A);
2. compare the oracle's samples, fine and coarse, with those exact per-level laws
   (Kolmogorov-Smirnov and moments);
3. check the OU velocity law without walls (exact at grid points for the O-step,
   Sec. 3.1);
4. check the exact identity that the GL/BAOAB coupling of Eq. (19), with the sign
   factors of Eq. (32), implies: fine and coarse extended velocities coincide at
   coarse times, so U_f(T)^2 = U_c(T)^2 sample by sample even through reflections,
   and the naive coupling (all S = 1) breaks it.
"""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.special import ndtr

import workloads as W

H = 1000.0


def chain_law(integ, sigma_u, tau, h, M, x0, u_mean, u_var):
    """Mean and covariance of the free (unreflected) linear Gaussian chain (U, X)."""
    lam = 1.0 / tau
    if integ == "SE":
        rho, s = 1.0 - lam * h, sigma_u * math.sqrt(2.0 * lam * h)
        A = np.array([[rho, 0.0], [h * rho, 1.0]]); b = np.array([s, h * s])
    elif integ == "GL":
        rho, s = math.exp(-lam * h), sigma_u * math.sqrt(-math.expm1(-2.0 * lam * h))
        A = np.array([[rho, 0.0], [h * rho, 1.0]]); b = np.array([s, h * s])
    else:
        rho, s = math.exp(-lam * h), sigma_u * math.sqrt(-math.expm1(-2.0 * lam * h))
        A = np.array([[rho, 0.0], [0.5 * h * (1.0 + rho), 1.0]]); b = np.array([s, 0.5 * h * s])
    m = np.array([u_mean, x0]); Cv = np.array([[u_var, 0.0], [0.0, 0.0]])
    for _ in range(M):
        m = A @ m
        Cv = A @ Cv @ A.T + np.outer(b, b)
    return m, Cv


def fold_cdf(x, mu, sd, kmax=60):
    """P(fold(Z) <= x), Z ~ N(mu, sd^2), fold onto [0, H] by reflections at 0 and H."""
    k = np.arange(-kmax, kmax + 1)[:, None]
    x = np.atleast_1d(x)[None, :]
    return np.sum(ndtr((2 * k * H + x - mu) / sd) - ndtr((2 * k * H - x - mu) / sd), axis=0)


def fold_mean(mu, sd):
    xs = np.linspace(0.0, H, 20001)
    return np.trapezoid(1.0 - fold_cdf(xs, mu, sd), xs)


def continuous_mean_var(sigma_u, tau, T, x0, w0=None):
    """Integrated OU position: stationary start (w0 None) or fixed velocity w0."""
    if w0 is None:
        return x0, 2 * sigma_u**2 * tau**2 * (T / tau - 1 + math.exp(-T / tau))
    r = T / tau
    return (x0 + w0 * tau * (1 - math.exp(-r)),
            sigma_u**2 * tau**2 * (2 * r - 3 + 4 * math.exp(-r) - math.exp(-2 * r)))


@pytest.mark.parametrize("integ,order", [("SE", 1), ("GL", 1), ("BAOAB", 2)])
def test_discrete_laws_converge_at_paper_orders(integ, order):
    """Release at 100 m with w0 = 0 (a case with a large bias): E[Z_l] -> E[Z] with
    error ratio 2^order between successive levels."""
    mu_c, var_c = continuous_mean_var(1.3, 100.0, 1000.0, 100.0, 0.0)
    exact = fold_mean(mu_c, math.sqrt(var_c))
    errs = []
    for l in range(8):
        M = 8 << l
        m, Cv = chain_law(integ, 1.3, 100.0, 1000.0 / M, M, 100.0, 0.0, 0.0)
        errs.append(fold_mean(m[1], math.sqrt(Cv[1, 1])) - exact)
    ratios = np.array(errs[3:-1]) / np.array(errs[4:])
    assert np.all(np.abs(ratios - 2.0**order) < 0.1 * 2.0**order), ratios


def _level_law(p, integ, level):
    M = p["M0"] << level
    if p["release"] == "gaussian":
        um, uv = 0.0, p["sigma_u"] ** 2
    else:
        um, uv = p["w0"], 0.0
    return chain_law(integ, p["sigma_u"], p["tau"], p["T"] / M, M, p["z0"], um, uv)


@pytest.mark.parametrize("integ", ["SE", "GL", "BAOAB"])
@pytest.mark.parametrize("release", ["gaussian", "fixed"])
def test_oracle_samples_follow_exact_level_laws(orc, integ, release):
    p = W.homogeneous(integrator=integ, release=release, z0=100.0 if release == "fixed" else 500.0)
    n = 20000
    for level in range(0, 4):
        st = orc.level_states(p, level, 0, n)
        paths = [(st[:, 0], st[:, 1], level)]
        if level > 0:
            paths.append((st[:, 2], st[:, 3], level - 1))   # coarse path ~ level l-1 law
        for xs, us, lev in paths:
            m, Cv = _level_law(p, integ, lev)
            mu, sd = m[1], math.sqrt(Cv[1, 1])
            ks = stats.kstest(xs, lambda x: fold_cdf(x, mu, sd))
            assert ks.pvalue > 1e-4, (level, lev, ks)
            assert abs(xs.mean() - fold_mean(mu, sd)) < 4.5 * xs.std() / math.sqrt(n)
            # reflection flips U's sign but keeps U^2: E[U^2] = Var + mean^2 of the chain
            eu2 = Cv[0, 0] + m[0] ** 2
            assert abs((us**2).mean() - eu2) < 4.5 * (us**2).std() / math.sqrt(n)


@pytest.mark.parametrize("integ", ["GL", "BAOAB"])
def test_ou_velocity_without_walls_is_exact(orc, integ):
    """GL and BAOAB integrate the OU part exactly (Sec. 3.1), so at any h:
    E[W_T] = w0 e^{-T/tau}, E[W_T^2] = w0^2 e^{-2T/tau} + sigma^2 (1 - e^{-2T/tau})."""
    sig, tau, T, w0 = 1.3, 100.0, 1000.0, 5.0
    n = 50000
    for qoi, exact in [("velocity", w0 * math.exp(-T / tau)),
                       ("velocity_sq", w0**2 * math.exp(-2 * T / tau) + sig**2 * (1 - math.exp(-2 * T / tau)))]:
        p = W.homogeneous(integrator=integ, H=1e12, z0=5e11, release="fixed", w0=w0, qoi=qoi)
        for level in (0, 2):
            s = orc.level_sums(p, level, 0, n)
            mean = s["sum_pf"] / n
            sd = math.sqrt(s["sum_pf2"] / n - mean**2)
            assert abs(mean - exact) < 4.5 * sd / math.sqrt(n), (qoi, level, mean, exact)


@pytest.mark.parametrize("integ", ["GL", "BAOAB"])
def test_coupled_extended_velocities_coincide(orc, integ):
    """Eq. (19) with the sign factors of Eq. (32): U_f(T)^2 == U_c(T)^2 per sample."""
    p = W.homogeneous(integrator=integ, qoi="velocity_sq")
    for level in (1, 3):
        pf_pc = orc.level_samples(p, level, 0, 4000)
        err = np.abs(pf_pc[:, 0] - pf_pc[:, 1]) / (pf_pc[:, 0] + 1.69)
        assert err.max() < 1e-12
        # positions differ (the A-steps see different velocities) and paths do reflect
        st = orc.level_states(W.homogeneous(integrator=integ), level, 0, 4000)
        assert np.mean(np.abs(st[:, 0] - st[:, 2]) > 1e-3) > 0.5
    naive = orc.level_samples(dict(p, coupling="naive"), 3, 0, 4000)
    assert np.mean(np.abs(naive[:, 0] - naive[:, 1]) > 1e-6 * (naive[:, 0] + 1.69)) > 0.3


@pytest.mark.parametrize("integ", ["GL", "BAOAB"])
def test_coupled_velocity_without_walls_coincides(orc, integ):
    """Without walls the signed velocities coincide (weight e^{-lambda h} of Eq. 19)."""
    p = W.homogeneous(integrator=integ, H=1e12, z0=5e11, qoi="velocity")
    pf_pc = orc.level_samples(p, 2, 0, 4000)
    assert np.max(np.abs(pf_pc[:, 0] - pf_pc[:, 1])) < 1e-12 * 10


def test_se_brownian_bridge_increment_without_walls(orc):
    """SE coupling of Eq. (18): with tau -> infinity and no walls the velocity is
    sigma sqrt(h) times the sum of the normals, the same for both paths."""
    p = W.homogeneous(integrator="SE", H=1e12, z0=5e11, tau=1e200, sigma_u=1e100,
                      qoi="velocity", release="fixed", w0=0.0)
    pf_pc = orc.level_samples(p, 3, 0, 2000)
    sig = math.sqrt(2 * 1e200 / 1e200)      # sigma = sqrt(2 sigma_U^2 / tau) = sqrt(2)
    assert np.allclose(pf_pc[:, 0], pf_pc[:, 1], rtol=1e-12, atol=1e-12 * sig)
    # and U_T ~ N(0, sigma^2 T)
    assert stats.kstest(pf_pc[:, 0] / (sig * math.sqrt(1000.0)), "norm").pvalue > 1e-4
