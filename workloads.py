"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module only produces parameters (plain dicts of numbers and names, SI units)
and seeded random parameter draws; it holds none of the method's arithmetic. Both
the GPU binding and the oracle binding marshal these dicts into their own structs.

Physical parameters follow the paper (Sec. 6): kappa_sigma = 1.3, kappa_tau = 0.5,
u_* = 0.2 m/s, H = 1 km, eps_reg = 0.01 H; the paper's reference set-up releases at
X_0 = 0.05 H with U_0 = 0.1 m/s and runs to T = 1000 s with M_0 = 40.
"""
from __future__ import annotations

import numpy as np

NEUTRAL = dict(profile="neutral", H=1000.0, sigma_u=0.0, tau=0.0, kappa_sigma=1.3,
               kappa_tau=0.5, u_star=0.2, eps_reg=10.0)


def problem(**kw) -> dict:
    """Default: neutral boundary layer, paper release (50 m, 0.1 m/s), BAOAB, E[X_T]."""
    p = dict(NEUTRAL)
    p.update(release="fixed", z0=50.0, w0=0.1, qoi="mean_z", qa=0.0, qb=0.0, r=0,
             delta=100.0, T=1000.0, M0=40, seed=42, stream_id=0, integrator="BAOAB")
    p.update(kw)
    return p


def homogeneous(**kw) -> dict:
    """Homogeneous turbulence (OU velocity): sigma_w = 1.3 m/s, tau = 100 s, H = 1 km,
    release at 500 m with w0 ~ N(0, sigma^2), T = 1000 s, M_0 = 8, SE, E[Z(T)], seed 42."""
    p = problem(profile="homogeneous", sigma_u=1.3, tau=100.0, kappa_sigma=0.0,
                kappa_tau=0.0, u_star=0.0, eps_reg=0.0, release="gaussian", z0=500.0,
                w0=0.0, M0=8, integrator="SE")
    p.update(kw)
    return p


def neutral(z0=500.0, integrator="BAOAB", **kw) -> dict:
    """Neutral boundary layer released at z0 with w0 ~ N(0, sigma_U(z0)^2), M_0 = 40."""
    p = problem(release="gaussian", z0=float(z0), w0=0.0, integrator=integrator, M0=40)
    p.update(kw)
    return p


def well_mixed(integrator="BAOAB", **kw) -> dict:
    """Particles uniform on [0, H] with U_0 ~ N(0, sigma_U(X_0)^2); phi = X_T."""
    p = problem(release="well_mixed", z0=0.0, w0=0.0, integrator=integrator, M0=40)
    p.update(kw)
    return p


def single_large(integrator="BAOAB", **kw) -> dict:
    """The large single estimate: neutral layer, release at 500 m with Gaussian w0,
    T = 1000 s, dt_0 = T/8, levels 0..12, relative eps 1e-4, E[Z(T)]."""
    p = neutral(500.0, integrator, M0=8)
    p.update(kw)
    return p


SINGLE_LARGE_LEVELS = 12
SINGLE_LARGE_EPS_REL = 1e-4

# Level-0..4 homogeneous case: 10^4 coupled samples per level.
HOMOGENEOUS_LEVELS = 4
HOMOGENEOUS_N = 10_000


def batched_estimators(n: int = 64, seed: int = 7, eps_range=(1e-3, 1e-2)) -> list:
    """n independent estimators: release height U[50, 950] m, eps log-uniform in
    eps_range, integrator uniform over the three, QoI E[Z(T)] or P(Z(T) > z*) with
    z* ~ U[200, 800] m (smoothed, r = 4, delta = 100 m). The tolerance is relative for
    E[Z(T)] and absolute (probability units) for P(Z(T) > z*): such probabilities can
    be 1e-6 or smaller (release low, threshold high), and a relative tolerance there
    asks for more than 1e11 samples."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        z0 = float(rng.uniform(50.0, 950.0))
        eps = float(np.exp(rng.uniform(np.log(eps_range[0]), np.log(eps_range[1]))))
        integ = ["SE", "GL", "BAOAB"][int(rng.integers(0, 3))]
        if rng.uniform() < 0.5:
            q = dict(qoi="mean_z")
        else:
            q = dict(qoi="p_above", qa=float(rng.uniform(200.0, 800.0)), r=4, delta=100.0)
        out.append(dict(problem=neutral(z0, integ, seed=1000 + k, stream_id=k, **q),
                        eps=eps, eps_is_relative=q["qoi"] == "mean_z"))
    return out


def poisson_arrivals(rate: float, duration: float, seed: int = 11,
                     eps_range=(3e-4, 1e-2)) -> list:
    """Arrival times of a Poisson process and the query parameters of each arrival."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        k = len(out)
        q = batched_estimators(1, seed=seed * 100003 + k, eps_range=eps_range)[0]
        q["problem"]["stream_id"] = k % (1 << 24)
        q["arrival"] = t
        out.append(q)
    return out
