"""GPU tests of the early top-up schedule of mlmc_estimate (ld_estimate_opts.early_topup).

The short levels' first batch runs beside the long levels' on a second stream and part of
their top-up is drawn before the long levels end. The draws are the same as in the plain
schedule (indices from 0 on every level), so:
- the FP64 estimate equals the oracle's MLMC estimate over the same N_l (sums over
  [0, N_l) on every level, recomputed on the CPU) within 1e-11;
- the run is deterministic (two calls agree bit for bit);
- it converges like the plain schedule, to an estimate within the statistical error, and
  draws between 0.9 and 1.25 times the plain schedule's samples on the short levels (the
  long levels' share of the variance rule is extrapolated, and each count carries a
  margin of three standard errors of its variance estimate: 1.095 at N_init = 2000);
- too few levels (L0 < 5) and fixed_N fall back to the plain schedule exactly.
"""
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


CFG = W.single_large("BAOAB")
KW = dict(fixed_L=7, eps_is_relative=True, N_init=2000)


def test_fp64_estimate_equals_oracle_over_the_same_samples():
    say("early top-up FP64, levels 0..7, eps_rel 1e-3")
    g = ld.estimate(1e-3, CFG, precision="fp64", early_topup=True, **KW)
    assert g["status"] == 1 and g["launches"] >= 3
    est = 0.0
    for l, n in enumerate(g["N"]):
        s = oracle.level_sums(CFG, l, 0, n)
        est += s["sum_y"] / s["n"]
    say(f"  N={g['N']} estimate {g['estimate']:.9f} oracle {est:.9f}")
    assert abs(g["estimate"] - est) <= 1e-11 * abs(est)


def test_deterministic_and_consistent_with_the_plain_schedule():
    a = ld.estimate(1e-3, CFG, precision="fp32", early_topup=True, **KW)
    b = ld.estimate(1e-3, CFG, precision="fp32", early_topup=True, **KW)
    assert a["N"] == b["N"] and a["estimate"] == b["estimate"]
    p = ld.estimate(1e-3, CFG, precision="fp32", **KW)
    say(f"  early N={a['N']} plain N={p['N']}")
    assert a["status"] == p["status"] == 1
    assert a["rmse_est"] <= 1e-3 * abs(a["estimate"]) * 1.01
    assert abs(a["estimate"] - p["estimate"]) <= 3.0 * np.sqrt(a["stat_var"] + p["stat_var"])
    for l in range(3):                      # short levels 0..L0-5
        assert 0.9 * p["N"][l] - 1 <= a["N"][l] <= 1.25 * p["N"][l] + 1


def test_falls_back_to_the_plain_schedule():
    for kw in (dict(fixed_L=4, eps_is_relative=True, N_init=2000),
               dict(fixed_L=7, fixed_N=True, eps_is_relative=True, N_init=500)):
        a = ld.estimate(1e-3, CFG, precision="fp64", early_topup=True, **kw)
        b = ld.estimate(1e-3, CFG, precision="fp64", **kw)
        assert a["N"] == b["N"] and a["estimate"] == b["estimate"]


def test_adaptive_problem_with_early_topup_equals_oracle():
    """Adaptive symplectic Euler (Sec. 7) through the early top-up schedule: the FP64
    estimate equals the oracle's MLMC estimate over the same N_l."""
    cfg = W.problem(integrator="SE", M0=40, x_adapt=50.0)
    g = ld.estimate(1e-2, cfg, precision="fp64", early_topup=True, fixed_L=5, eps_is_relative=True,
                    N_init=500)
    est = sum(s["sum_y"] / s["n"] for s in (oracle.level_sums(cfg, l, 0, n) for l, n in enumerate(g["N"])))
    say(f"  adaptive early top-up N={g['N']} {g['estimate']:.9f} oracle {est:.9f}")
    assert abs(g["estimate"] - est) <= 1e-11 * abs(est)


def test_second_stream_waits_for_work_the_caller_queued_before():
    """The workspace may be memory that work still queued on the caller's stream reads
    (a caching allocator hands memory out again in stream order). Here a sum over the
    workspace buffer is queued behind a long chain of matrix products; the estimate that
    follows must not write the buffer before the sum has read it, on either of its two
    streams. The sum sees the buffer's old contents and the estimate equals a run on a
    fresh workspace bit for bit."""
    import torch
    ref = ld.estimate(1e-3, CFG, precision="fp32", early_topup=True, **KW)
    nbytes = ld.estimate_workspace_bytes()
    n = nbytes // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    a = torch.randn(4096, 4096, device="cuda")
    for _ in range(8):                       # some ms of queued work before the sum
        a = (a @ a) * (1.0 / 64.0)
    total = x.sum()
    got = ld.estimate(1e-3, CFG, precision="fp32", early_topup=True, workspace=x.view(torch.uint8), **KW)
    torch.cuda.synchronize()
    say(f"  sum before the estimate {total.item():.0f} of {n}")
    assert total.item() == float(n)
    assert got["N"] == ref["N"] and got["estimate"] == ref["estimate"]
