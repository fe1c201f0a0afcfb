"""Pins of the oracle's model functions and single integrator steps.

- the drift equals the X-derivative of the potential V printed after Eq. (3),
  differentiated numerically in 50-digit arithmetic (not the oracle's formula);
- the drift also equals the form of Eq. (3) with d sigma_U^2 / dX by numerical
  differentiation;
- the regularised tau never falls below ~19.4 s at eps_reg = 0.01 H, matching the
  20 s quoted in Sec. 6;
- the SE stability bound h < 2 / lambda of Sec. 3.1 reproduces the M_0 = 270 the
  paper needed at eps_reg = 0.001 H (Sec. 7.1);
- one step of each integrator against a 50-digit brute-force evaluation of
  Eqs. (8)-(10), including wall hits, double folds and the cut-off layers.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import workloads as W

mp.mp.dps = 50


def _sigma_u_mp(p, x):
    if p["profile"] == "homogeneous":
        return mp.mpf(p["sigma_u"])
    H, e = mp.mpf(p["H"]), mp.mpf(p["eps_reg"])
    xr = min(max(mp.mpf(x), e), H - e)          # Eq. (7)
    return mp.mpf(p["kappa_sigma"]) * mp.mpf(p["u_star"]) * (1 - xr / H) ** mp.mpf(0.75)


def _tau_mp(p, x):
    if p["profile"] == "homogeneous":
        return mp.mpf(p["tau"])
    H, e = mp.mpf(p["H"]), mp.mpf(p["eps_reg"])
    xr = min(max(mp.mpf(x), e), H - e)
    return mp.mpf(p["kappa_tau"]) * xr / _sigma_u_mp(p, x)


def _V_mp(p, x, u, xref=500):
    """The potential defined after Eq. (3)."""
    s2 = _sigma_u_mp(p, x) ** 2
    return -mp.mpf(1) / 2 * (s2 + mp.mpf(u) ** 2 * mp.log(s2 / _sigma_u_mp(p, xref) ** 2))


def _dVdX_mp(p, x, u):
    return mp.diff(lambda t: _V_mp(p, t, u), mp.mpf(x))


@pytest.mark.parametrize("x", [10.5, 37.0, 50.0, 123.4, 500.0, 871.0, 989.0])
@pytest.mark.parametrize("u", [0.0, 0.13, -0.7, 2.5])
def test_drift_is_derivative_of_printed_potential(orc, x, u):
    p = W.problem()
    ref = _dVdX_mp(p, x, u)
    got = orc.dVdX(p, x, u)
    assert abs(got - float(ref)) <= 1e-12 * max(abs(float(ref)), 1e-12)


@pytest.mark.parametrize("x", [50.0, 300.0, 900.0])
@pytest.mark.parametrize("u", [0.0, 0.4])
def test_drift_matches_thomson_form(orc, x, u):
    """-dV/dX = 1/2 [1 + (U/sigma_U)^2] d(sigma_U^2)/dX, the drift of Eq. (3)."""
    p = W.problem()
    ds2 = mp.diff(lambda t: _sigma_u_mp(p, t) ** 2, mp.mpf(x))
    drift = mp.mpf(1) / 2 * (1 + (mp.mpf(u) / _sigma_u_mp(p, x)) ** 2) * ds2
    assert abs(-orc.dVdX(p, x, u) - float(drift)) <= 1e-12 * abs(float(drift))


@pytest.mark.parametrize("x", [0.0, 3.0, 9.999, 990.01, 999.0, 1000.0])
def test_drift_vanishes_in_cutoff_layers(orc, x):
    p = W.problem()
    assert orc.dVdX(p, x, 0.3) == 0.0
    assert orc.profile(p, x) in (orc.profile(p, 10.0), orc.profile(p, 990.0))


def test_homogeneous_profile_is_constant(orc):
    p = W.homogeneous()
    for x in (0.0, 1.0, 500.0, 1000.0):
        assert orc.profile(p, x) == (1.3, 100.0)
        assert orc.dVdX(p, x, 1.0) == 0.0


def test_tau_floor_matches_paper(orc):
    """Sec. 6: with eps_reg = 0.01 H the decorrelation time stays at the ~20 s quoted
    (the regularised minimum tau(eps_reg) = 19.4 s)."""
    p = W.problem()
    taus = [orc.profile(p, x)[1] for x in np.linspace(0, 1000, 2001)]
    assert min(taus) == pytest.approx(orc.profile(p, 10.0)[1])
    assert 19.0 < min(taus) < 20.0


def test_se_stability_bound_matches_paper_m0():
    """Sec. 3.1: SE needs h < 2 / lambda. Sec. 6 uses M_0 = 40 at eps_reg = 10 m;
    Sec. 7.1 needs M_0 = 270 at eps_reg = 1 m for stability on all levels."""
    p = W.problem()
    lam10 = 1.0 / float(_tau_mp(p, 10.0))
    assert math.ceil(p["T"] / (2 / lam10)) == 26 <= 40
    lam1 = 1.0 / float(_tau_mp(dict(p, eps_reg=1.0), 1.0))
    m0_min = math.ceil(p["T"] / (2 / lam1))
    assert 200 < m0_min <= 270


# --------------------------------------------------------------------------- steps
def _fold_mp(H, x, u, s):
    while x < 0 or x > H:
        x = -x if x < 0 else 2 * H - x
        u, s = -u, -s
    return x, u, s


def _step_mp(p, h, x, u, s, xi, tilde_in):
    """Eqs. (8)-(10) in 50 digits, written in the paper's literal form."""
    h, x, u, xi = mp.mpf(h), mp.mpf(x), mp.mpf(u), mp.mpf(xi)
    H = mp.mpf(p["H"])
    lam = lambda t: 1 / _tau_mp(p, t)
    sig = lambda t: mp.sqrt(2 * _sigma_u_mp(p, t) ** 2 / _tau_mp(p, t))

    def dV(t, v):
        if p["profile"] == "homogeneous":
            return mp.mpf(0)
        e = mp.mpf(p["eps_reg"])
        if t < e or t > H - e:
            return mp.mpf(0)
        return _dVdX_mp(p, t, v)

    def phys(sign):
        return sign * xi if tilde_in else xi

    if p["integrator"] == "SE":
        noise = phys(s)
        tilde = s * noise
        l = lam(x)
        u1 = (1 - l * h) * u - dV(x, u) * h + sig(x) * mp.sqrt(h) * noise
        x1 = x + u1 * h
        x1, u1, s = _fold_mp(H, x1, u1, s)
        return x1, u1, s, tilde, l
    if p["integrator"] == "GL":
        noise = phys(s)
        tilde = s * noise
        l = lam(x)
        us = mp.e ** (-l * h) * u + sig(x) * mp.sqrt((1 - mp.e ** (-2 * l * h)) / (2 * l)) * noise
        u1 = us - dV(x, us) * h
        x1 = x + u1 * h
        x1, u1, s = _fold_mp(H, x1, u1, s)
        return x1, u1, s, tilde, l
    uh = u - dV(x, u) * h / 2
    xh = x + uh * h / 2
    xh, uh, s = _fold_mp(H, xh, uh, s)
    noise = phys(s)
    tilde = s * noise
    l = lam(xh)
    us = mp.e ** (-l * h) * uh + sig(xh) * mp.sqrt((1 - mp.e ** (-2 * l * h)) / (2 * l)) * noise
    x1 = xh + us * h / 2
    x1, us, s = _fold_mp(H, x1, us, s)
    u1 = us - dV(x1, us) * h / 2
    return x1, u1, s, tilde, l


_CASES = [
    # (profile, h, x, u, s, xi)
    ("neutral", 25.0, 50.0, 0.1, 1.0, 0.3),
    ("neutral", 25.0, 400.0, -0.2, -1.0, -1.7),
    ("neutral", 3.125, 12.0, -0.5, 1.0, 0.1),       # hits the ground
    ("neutral", 25.0, 5.0, 0.05, 1.0, 2.0),         # inside the lower cut-off layer
    ("neutral", 25.0, 995.0, 0.02, -1.0, -0.4),     # inside the upper cut-off layer
    ("neutral", 25.0, 985.0, 0.3, 1.0, 0.9),        # hits the top
    ("neutral", 0.78125, 700.0, 0.15, 1.0, -2.2),
    ("homogeneous", 125.0, 100.0, -3.0, 1.0, 0.5),  # double fold
    ("homogeneous", 125.0, 900.0, 9.0, -1.0, -0.2), # several folds through the top
    ("homogeneous", 7.8125, 500.0, 1.0, 1.0, 0.0),
]


@pytest.mark.parametrize("integ", ["SE", "GL", "BAOAB"])
@pytest.mark.parametrize("case", _CASES)
@pytest.mark.parametrize("tilde_in", [False, True])
def test_single_step_brute_force(orc, integ, case, tilde_in):
    prof, h, x, u, s, xi = case
    p = W.problem(integrator=integ) if prof == "neutral" else W.homogeneous(integrator=integ)
    st, tilde, lam_o, rc = orc.step(p, h, [x, u, s], xi, noise_is_tilde=tilde_in)
    x1, u1, s1, t1, l1 = _step_mp(p, h, x, u, s, xi, tilde_in)
    assert rc == 0
    assert st[2] == float(s1)
    assert abs(st[0] - float(x1)) <= 1e-12 * max(abs(float(x1)), 1.0)
    assert abs(st[1] - float(u1)) <= 1e-12 * max(abs(float(u1)), 1e-3)
    assert tilde == float(t1)
    assert lam_o == pytest.approx(float(l1), rel=1e-14)


def test_fold_edge_semantics(orc):
    """0 and H are inside the domain; a position outside is folded back (Eq. 6)."""
    p = W.homogeneous(integrator="SE", tau=1e300)      # no damping, no drift, xi = 0
    st, _, _, _ = orc.step(p, 1.0, [0.5, -0.5, 1.0], 0.0)
    assert st == [0.0, -0.5, 1.0]                      # lands exactly on 0: no fold
    st, _, _, _ = orc.step(p, 1.0, [999.0, 1.0, 1.0], 0.0)
    assert st == [1000.0, 1.0, 1.0]                    # lands exactly on H: no fold
    st, _, _, _ = orc.step(p, 1.0, [0.25, -0.5, 1.0], 0.0)
    assert st == [0.25, 0.5, -1.0]
    st, _, _, _ = orc.step(p, 1.0, [500.0, 2600.0, 1.0], 0.0)   # 3100 -> -1100 -> 1100 -> 900
    assert st[0] == 900.0 and st[1] == -2600.0 and st[2] == -1.0


def test_runaway_step_is_marked_nonfinite(orc):
    p = W.homogeneous(integrator="SE", tau=1e300)
    st, _, _, rc = orc.step(p, 1.0, [500.0, 1e9, 1.0], 0.0)
    assert rc != 0 and math.isnan(st[0])


@pytest.mark.parametrize("z0", [30.0, 500.0, 900.0])
def test_gaussian_release_follows_conditional_velocity_law(orc, z0):
    """The Gaussian release draws U_0 from the conditional law of the well-mixed
    condition (Sec. 2): N(0, sigma_U(z0)^2). Over a vanishing T the terminal velocity
    is U_0."""
    from scipy import stats
    p = W.neutral(z0, "GL", T=1e-9, M0=1, qoi="velocity")
    u0 = orc.level_samples(p, 0, 0, 20000)[:, 0]
    su = float(_sigma_u_mp(p, z0))
    assert stats.kstest(u0 / su, "norm").pvalue > 1e-4


def test_raw_indicators_follow_definition(orc):
    """Eq. (34): 1_[a,b](X) = theta(X - b) - theta(X - a) with theta(s) = 1 for s <= 0,
    i.e. 1 on (a, b]; and 1(X > z*) = 1 - theta(X - z*)."""
    box = W.problem(qoi="p_box", qa=105.5, qb=155.5, r=0)
    for x, want in [(0.0, 0.0), (105.5, 0.0), (105.6, 1.0), (130.0, 1.0), (155.5, 1.0),
                    (155.6, 0.0), (1000.0, 0.0)]:
        assert orc.qoi(box, x) == want, x
    above = W.problem(qoi="p_above", qa=400.0, r=0)
    for x, want in [(0.0, 0.0), (400.0, 0.0), (400.001, 1.0), (1000.0, 1.0)]:
        assert orc.qoi(above, x) == want, x
