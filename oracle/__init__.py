"""ctypes binding of the plain CPU FP64 oracle (oracle/oracle.c).

TEST INFRASTRUCTURE: only the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. The product library
(``paper_1612_07717_amd``) never imports it and shares no code with it.

Problems are plain dicts as produced by ``workloads.problem`` (SI units).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_DEFAULT_LIB = os.path.join(_HERE, "liboracle.so")
# A test that plants a mistake in a copy of the oracle points this at the copy.
_LIB_PATH = os.environ.get("LD_ORACLE_LIB", _DEFAULT_LIB)

INTEGRATORS = {"SE": 0, "GL": 1, "BAOAB": 2}
PROFILES = {"homogeneous": 0, "neutral": 1}
RELEASES = {"fixed": 0, "gaussian": 1, "well_mixed": 2}
QOIS = {"mean_z": 0, "p_above": 1, "p_box": 2, "velocity": 3, "velocity_sq": 4}
COUPLINGS = {"reflected": 0, "naive": 1}
MAX_LEVELS = 32


def build(src: str = _SRC, out: str = _DEFAULT_LIB, extra_flags=()) -> str:
    """Compile liboracle.so with gcc (FP64, no fast-math, no FMA contraction).
    `extra_flags` go to gcc as they are (a sanitizer build passes its options here)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra", *extra_flags,
           "-I", _HERE, "-o", out + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(out + ".tmp", out)
    return out


class Problem(C.Structure):
    _fields_ = [
        ("profile_kind", C.c_int32), ("integrator", C.c_int32),
        ("H", C.c_double), ("sigma_u", C.c_double), ("tau", C.c_double),
        ("kappa_sigma", C.c_double), ("kappa_tau", C.c_double),
        ("u_star", C.c_double), ("eps_reg", C.c_double),
        ("release_kind", C.c_int32), ("coupling", C.c_int32),
        ("z0", C.c_double), ("w0", C.c_double),
        ("qoi_kind", C.c_int32), ("r", C.c_int32),
        ("qa", C.c_double), ("qb", C.c_double), ("delta", C.c_double),
        ("T", C.c_double), ("M0", C.c_int32), ("stream_id", C.c_uint32),
        ("seed", C.c_uint64), ("x_adapt", C.c_double),
    ]


class Sums(C.Structure):
    _fields_ = [("s", C.c_double * 4), ("c", C.c_double * 4),
                ("n", C.c_uint64), ("n_nonfinite", C.c_uint64)]


class Opts(C.Structure):
    _fields_ = [("L_min", C.c_int32), ("L_max", C.c_int32), ("fixed_L", C.c_int32),
                ("fixed_N", C.c_int32), ("N_init", C.c_uint64),
                ("eps_is_relative", C.c_int32), ("max_iter", C.c_int32),
                ("alpha", C.c_double)]


class PlanIn(C.Structure):
    _fields_ = [("L", C.c_int32),
                ("n", C.c_uint64 * MAX_LEVELS),
                ("sum1", C.c_double * MAX_LEVELS), ("sum2", C.c_double * MAX_LEVELS),
                ("M0", C.c_int32), ("eps", C.c_double), ("eps_is_relative", C.c_int32),
                ("L_max", C.c_int32), ("fixed_L", C.c_int32), ("fixed_N", C.c_int32),
                ("N_init", C.c_uint64), ("alpha", C.c_double)]


class PlanOut(C.Structure):
    _fields_ = [("status", C.c_int32), ("L", C.c_int32),
                ("dn", C.c_uint64 * MAX_LEVELS),
                ("Yhat", C.c_double * MAX_LEVELS), ("V", C.c_double * MAX_LEVELS),
                ("estimate", C.c_double), ("eps_abs", C.c_double), ("alpha", C.c_double),
                ("bias_est", C.c_double), ("stat_var", C.c_double)]


class Result(C.Structure):
    _fields_ = [("estimate", C.c_double), ("eps_abs", C.c_double),
                ("bias_est", C.c_double), ("stat_var", C.c_double),
                ("rmse_est", C.c_double), ("alpha", C.c_double),
                ("L", C.c_int32), ("iterations", C.c_int32), ("status", C.c_int32),
                ("pad", C.c_int32),
                ("N", C.c_uint64 * MAX_LEVELS), ("n_nonfinite", C.c_uint64),
                ("Yhat", C.c_double * MAX_LEVELS), ("V", C.c_double * MAX_LEVELS),
                ("fine_steps", C.c_double), ("integrator_steps", C.c_double)]


_lib = None


MAX_LEVELS, MAX_BINS = 32, 64
MLMC, STMC = 0, 1


class PdfPlanIn(C.Structure):
    _fields_ = [("L", C.c_int32), ("n_bins", C.c_int32), ("n", C.c_uint64 * MAX_LEVELS),
                ("sum1", (C.c_double * MAX_BINS) * MAX_LEVELS),
                ("sum2", (C.c_double * MAX_BINS) * MAX_LEVELS),
                ("M0", C.c_int32), ("L_max", C.c_int32), ("eps", C.c_double),
                ("fixed_L", C.c_int32), ("pad", C.c_int32), ("N_init", C.c_uint64),
                ("alpha", C.c_double)]


class PdfPlanOut(C.Structure):
    _fields_ = [("status", C.c_int32), ("L", C.c_int32), ("dn", C.c_uint64 * MAX_LEVELS),
                ("V", C.c_double * MAX_LEVELS), ("estimate", C.c_double * MAX_BINS),
                ("bias_est", C.c_double), ("stat_var", C.c_double), ("alpha", C.c_double)]


class PdfResult(C.Structure):
    _fields_ = [("estimate", C.c_double * MAX_BINS), ("bias_est", C.c_double),
                ("stat_var", C.c_double), ("rmse_est", C.c_double), ("L", C.c_int32),
                ("iterations", C.c_int32), ("status", C.c_int32), ("estimator", C.c_int32),
                ("N", C.c_uint64 * MAX_LEVELS), ("n_nonfinite", C.c_uint64),
                ("V", C.c_double * MAX_LEVELS), ("fine_steps", C.c_double)]


def load():
    """Load liboracle.so, building it first if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = C.CDLL(_LIB_PATH)
    P = C.POINTER
    lib.oracle_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
    lib.oracle_normals.argtypes = [P(Problem), C.c_int32, C.c_uint64, C.c_uint32, P(C.c_double)]
    lib.oracle_profile.argtypes = [P(Problem), C.c_double, P(C.c_double), P(C.c_double)]
    lib.oracle_dVdX.argtypes = [P(Problem), C.c_double, C.c_double]
    lib.oracle_dVdX.restype = C.c_double
    lib.oracle_smoothing_poly.argtypes = [C.c_int32, P(C.c_double)]
    lib.oracle_qoi.argtypes = [P(Problem), C.c_double, C.c_double]
    lib.oracle_qoi.restype = C.c_double
    lib.oracle_step.argtypes = [P(Problem), C.c_double, P(C.c_double), C.c_double,
                                C.c_int32, P(C.c_double), P(C.c_double)]
    lib.oracle_sample.argtypes = [P(Problem), C.c_int32, C.c_uint64, P(C.c_double), P(C.c_double)]
    lib.oracle_level_samples.argtypes = [P(Problem), C.c_int32, C.c_uint64, C.c_uint64, P(C.c_double)]
    lib.oracle_level_states.argtypes = [P(Problem), C.c_int32, C.c_uint64, C.c_uint64, P(C.c_double)]
    lib.oracle_level_sums.argtypes = [P(Problem), C.c_int32, C.c_uint64, C.c_uint64, P(Sums)]
    lib.oracle_sums_value.argtypes = [P(Sums), C.c_int32]
    lib.oracle_sums_value.restype = C.c_double
    lib.oracle_plan.argtypes = [P(PlanIn), P(PlanOut)]
    lib.oracle_estimate.argtypes = [C.c_double, P(Problem), P(Opts), P(Result)]
    lib.oracle_pdf_level_sums.argtypes = [P(Problem), C.c_int32, C.c_uint64, C.c_uint64,
                                          C.c_double, C.c_double, C.c_int32, P(Sums)]
    lib.oracle_pdf_level_sums.restype = None
    lib.oracle_pdf_plan.argtypes = [P(PdfPlanIn), P(PdfPlanOut)]
    lib.oracle_pdf_plan.restype = None
    lib.oracle_estimate_pdf.argtypes = [C.c_double, P(Problem), P(Opts), C.c_double, C.c_double,
                                        C.c_int32, C.c_int32, P(PdfResult)]
    lib.oracle_num_threads.restype = C.c_int
    lib.oracle_set_num_threads.argtypes = [C.c_int]
    lib.oracle_set_num_threads.restype = None
    _lib = lib
    return lib


def make_problem(cfg: dict) -> Problem:
    """Marshal a workload dict into the oracle's problem struct."""
    p = Problem()
    p.profile_kind = PROFILES[cfg["profile"]]
    p.integrator = INTEGRATORS[cfg["integrator"]]
    for k in ("H", "sigma_u", "tau", "kappa_sigma", "kappa_tau", "u_star", "eps_reg",
              "z0", "w0", "qa", "qb", "delta", "T"):
        setattr(p, k, float(cfg[k]))
    p.release_kind = RELEASES[cfg["release"]]
    p.coupling = COUPLINGS[cfg.get("coupling", "reflected")]
    p.qoi_kind = QOIS[cfg["qoi"]]
    p.r = int(cfg["r"])
    p.M0 = int(cfg["M0"])
    p.stream_id = int(cfg["stream_id"])
    p.seed = int(cfg["seed"])
    p.x_adapt = float(cfg.get("x_adapt", 0.0))
    return p


def _sums_dict(s: Sums) -> dict:
    lib = load()
    vals = [lib.oracle_sums_value(C.byref(s), k) for k in range(4)]
    return {"sum_y": vals[0], "sum_y2": vals[1], "sum_pf": vals[2], "sum_pf2": vals[3],
            "s": list(s.s), "c": list(s.c), "n": int(s.n),
            "n_nonfinite": int(s.n_nonfinite)}


def philox(ctr, key):
    lib = load()
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib.oracle_philox4x32_10(c, k, o)
    return list(o)


def normals(cfg, level, sample, block):
    lib = load()
    p = make_problem(cfg)
    o = (C.c_double * 2)()
    lib.oracle_normals(C.byref(p), level, sample, block, o)
    return o[0], o[1]


def profile(cfg, x):
    lib = load()
    p = make_problem(cfg)
    su, tau = C.c_double(), C.c_double()
    lib.oracle_profile(C.byref(p), float(x), C.byref(su), C.byref(tau))
    return su.value, tau.value


def dVdX(cfg, x, u):
    return load().oracle_dVdX(C.byref(make_problem(cfg)), float(x), float(u))


def qoi(cfg, x, u=0.0):
    return load().oracle_qoi(C.byref(make_problem(cfg)), float(x), float(u))


def smoothing_poly(r):
    coef = (C.c_double * 10)()
    rc = load().oracle_smoothing_poly(int(r), coef)
    if rc != 0:
        raise ValueError(f"r={r} out of range")
    return np.array(coef[: r + 2])


def step(cfg, h, state, xi, noise_is_tilde=False):
    """One integrator step; returns (new_state, tilde, lambda_o, rc)."""
    lib = load()
    st = (C.c_double * 3)(*state)
    tilde, lam = C.c_double(), C.c_double()
    rc = lib.oracle_step(C.byref(make_problem(cfg)), float(h), st, float(xi),
                         int(bool(noise_is_tilde)), C.byref(tilde), C.byref(lam))
    return list(st), tilde.value, lam.value, rc


def sample(cfg, level, i):
    pf, pc = C.c_double(), C.c_double()
    bad = load().oracle_sample(C.byref(make_problem(cfg)), level, i, C.byref(pf), C.byref(pc))
    return pf.value, pc.value, bad


def level_samples(cfg, level, begin, n) -> np.ndarray:
    out = np.empty((n, 2), dtype=np.float64)
    load().oracle_level_samples(C.byref(make_problem(cfg)), level, begin, n,
                                out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def level_states(cfg, level, begin, n) -> np.ndarray:
    out = np.empty((n, 4), dtype=np.float64)
    load().oracle_level_states(C.byref(make_problem(cfg)), level, begin, n,
                               out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def level_sums(cfg, level, begin, n) -> dict:
    s = Sums()
    load().oracle_level_sums(C.byref(make_problem(cfg)), level, begin, n, C.byref(s))
    return _sums_dict(s)


def plan(d: dict) -> dict:
    """One decision of the oracle's adaptive MLMC algorithm."""
    pin = PlanIn()
    pin.L = d["L"]
    for l, v in enumerate(d["n"]):
        pin.n[l] = int(v)
    for l, v in enumerate(d["sum1"]):
        pin.sum1[l] = float(v)
    for l, v in enumerate(d["sum2"]):
        pin.sum2[l] = float(v)
    pin.M0 = d["M0"]
    pin.eps = d["eps"]
    pin.eps_is_relative = int(d.get("eps_is_relative", 0))
    pin.L_max = d.get("L_max", 20)
    pin.fixed_L = d.get("fixed_L", -1)
    pin.fixed_N = int(d.get("fixed_N", 0))
    pin.N_init = d.get("N_init", 10000)
    pin.alpha = d.get("alpha", 1.0)
    out = PlanOut()
    load().oracle_plan(C.byref(pin), C.byref(out))
    Lp = out.L
    return {"status": out.status, "L": Lp, "dn": [int(out.dn[l]) for l in range(Lp + 1)],
            "Yhat": list(out.Yhat[: d["L"] + 1]), "V": list(out.V[: d["L"] + 1]),
            "estimate": out.estimate, "eps_abs": out.eps_abs, "alpha": out.alpha,
            "bias_est": out.bias_est, "stat_var": out.stat_var}


def estimate(eps, cfg, *, L_min=2, L_max=10, fixed_L=-1, fixed_N=False, N_init=10000,
             eps_is_relative=False, max_iter=100, alpha=1.0) -> dict:
    o = Opts(L_min=L_min, L_max=L_max, fixed_L=fixed_L, fixed_N=int(bool(fixed_N)),
             N_init=N_init, eps_is_relative=int(bool(eps_is_relative)), max_iter=max_iter,
             alpha=alpha)
    r = Result()
    rc = load().oracle_estimate(float(eps), C.byref(make_problem(cfg)), C.byref(o), C.byref(r))
    L = r.L
    return {"rc": rc, "estimate": r.estimate, "eps_abs": r.eps_abs, "bias_est": r.bias_est,
            "stat_var": r.stat_var, "rmse_est": r.rmse_est, "alpha": r.alpha, "L": L,
            "iterations": r.iterations, "status": r.status,
            "N": [int(r.N[l]) for l in range(L + 1)], "n_nonfinite": int(r.n_nonfinite),
            "Yhat": list(r.Yhat[: L + 1]), "V": list(r.V[: L + 1]),
            "fine_steps": r.fine_steps, "integrator_steps": r.integrator_steps}


def pdf_level_sums(cfg, level, begin, n, a0, width, n_bins) -> list:
    """Per-bin sums of the binned concentration (Sec. 6.4), one dict per bin."""
    out = (Sums * n_bins)()
    load().oracle_pdf_level_sums(C.byref(make_problem(cfg)), level, begin, n, float(a0),
                                 float(width), n_bins, out)
    return [_sums_dict(s) for s in out]


def pdf_plan(d: dict) -> dict:
    """d: L, n_bins, n[l], sum1[l][i], sum2[l][i], M0, eps, L_max, fixed_L, N_init, alpha."""
    pin = PdfPlanIn()
    pin.L, pin.n_bins = d["L"], d["n_bins"]
    for l in range(d["L"] + 1):
        pin.n[l] = d["n"][l]
        for i in range(d["n_bins"]):
            pin.sum1[l][i] = d["sum1"][l][i]
            pin.sum2[l][i] = d["sum2"][l][i]
    pin.M0, pin.eps, pin.L_max = d["M0"], d["eps"], d.get("L_max", 20)
    pin.fixed_L, pin.N_init, pin.alpha = d.get("fixed_L", -1), d.get("N_init", 10000), d.get("alpha", 1.0)
    out = PdfPlanOut()
    load().oracle_pdf_plan(C.byref(pin), C.byref(out))
    L = out.L
    return {"status": out.status, "L": L, "dn": [int(out.dn[l]) for l in range(L + 1)],
            "V": list(out.V[: d["L"] + 1]), "estimate": list(out.estimate[: d["n_bins"]]),
            "bias_est": out.bias_est, "stat_var": out.stat_var, "alpha": out.alpha}


def estimate_pdf(eps, cfg, a0, width, n_bins, *, estimator=MLMC, L_min=2, L_max=10, fixed_L=-1,
                 N_init=10000, max_iter=100, alpha=1.0) -> dict:
    o = Opts(L_min=L_min, L_max=L_max, fixed_L=fixed_L, fixed_N=0, N_init=N_init,
             eps_is_relative=0, max_iter=max_iter, alpha=alpha)
    r = PdfResult()
    rc = load().oracle_estimate_pdf(float(eps), C.byref(make_problem(cfg)), C.byref(o), float(a0),
                                    float(width), n_bins, estimator, C.byref(r))
    L = r.L
    nl = 1 if estimator == STMC else L + 1
    return {"rc": rc, "estimate": list(r.estimate[:n_bins]), "bias_est": r.bias_est,
            "stat_var": r.stat_var, "rmse_est": r.rmse_est, "L": L, "iterations": r.iterations,
            "status": r.status, "N": [int(r.N[l]) for l in range(nl)],
            "n_nonfinite": int(r.n_nonfinite), "V": list(r.V[:nl]), "fine_steps": r.fine_steps}


def num_threads() -> int:
    return int(load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of later oracle calls; the results do not depend on it."""
    load().oracle_set_num_threads(int(n))
