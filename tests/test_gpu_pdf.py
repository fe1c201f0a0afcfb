"""GPU tests of the binned concentration (vector QoI, Sec. 6.4) against the oracle.

- per-bin FP64 sums equal the oracle's within 1e-12 (same draws), on several levels,
  raw and smoothed boxes, ragged sample counts, and level 0 (no coarse path);
- one bin equals the scalar box QoI of the level kernels;
- FP32 paths give per-bin means within the statistical error of FP64 paths;
- the FP64 MLMC and StMC estimates take the oracle driver's decisions (same N_l) and
  agree per bin within 1e-11;
- a range longer than one dump chunk gives the same sums as one call over the range.
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


def _close(a, b, rel=1e-12):
    scale = max(abs(a), abs(b), 1e-300)
    return abs(a - b) <= rel * scale + 1e-12


CASES = [
    ("GL", 0, 4, 3000, 0.0, 50.0, 20),
    ("BAOAB", 2, 0, 2500, 0.0, 50.0, 20),
    ("SE", 3, 4, 1537, 100.0, 75.0, 9),
    ("BAOAB", 5, 4, 777, 0.0, 100.0, 10),
    ("GL", 1, 4, 4100, 0.0, 15.625, 64),
]


@pytest.mark.parametrize("integ,level,r,n,a0,w,k", CASES)
def test_pdf_sums_fp64_match_oracle(integ, level, r, n, a0, w, k):
    cfg = W.neutral(250.0, integ, r=r, delta=100.0)
    say(f"pdf sums {integ} level {level} r={r} n={n} bins={k}")
    g = ld.pdf_level_sums(cfg, level, 11, n, a0, w, k, precision="fp64")
    o = oracle.pdf_level_sums(cfg, level, 11, n, a0, w, k)
    for i, (x, y) in enumerate(zip(g, o)):
        assert x["n"] == y["n"] and x["n_nonfinite"] == y["n_nonfinite"], i
        for key in ("sum_y", "sum_y2", "sum_pf", "sum_pf2"):
            assert _close(x[key], y[key]), (i, key, x[key], y[key])


def test_one_bin_equals_the_scalar_box():
    cfg = W.neutral(400.0, "BAOAB", r=4, delta=100.0)
    g = ld.pdf_level_sums(cfg, 2, 0, 5000, 350.0, 50.0, 1, precision="fp64")[0]
    s = ld.level_sums(dict(cfg, qoi="p_box", qa=350.0, qb=400.0), 2, 0, 5000, precision="fp64")
    assert g["n"] == s["n"]
    for key in ("sum_y", "sum_y2", "sum_pf", "sum_pf2"):
        assert _close(g[key], s[key]), key


def test_fp32_bins_within_statistical_error_of_fp64():
    cfg = W.neutral(150.0, "GL", r=4, delta=100.0)
    n = 200000
    a = ld.pdf_level_sums(cfg, 3, 0, n, 0.0, 50.0, 20, precision="fp32")
    b = ld.pdf_level_sums(cfg, 3, 0, n, 0.0, 50.0, 20, precision="fp64")
    for x, y in zip(a, b):
        m32, m64 = x["sum_pf"] / x["n"], y["sum_pf"] / y["n"]
        sd = np.sqrt(max(y["sum_pf2"] / y["n"] - m64 * m64, 1e-12) / y["n"])
        assert abs(m32 - m64) <= 0.1 * sd + 1e-7, (m32, m64, sd)
        d32, d64 = x["sum_y"] / x["n"], y["sum_y"] / y["n"]
        sdy = np.sqrt(max(y["sum_y2"] / y["n"] - d64 * d64, 1e-14) / y["n"])
        assert abs(d32 - d64) <= 0.1 * sdy + 1e-7


@pytest.mark.parametrize("estimator", ["mlmc", "stmc"])
def test_fp64_pdf_estimate_matches_oracle_driver(estimator):
    cfg = W.neutral(200.0, "GL", r=4, delta=100.0, M0=80)
    kw = dict(N_init=2000, L_max=8)
    if estimator == "stmc":
        kw["fixed_L"] = 3
    g = ld.estimate_pdf(4e-3, cfg, 0.0, 100.0, 10, estimator=estimator, precision="fp64", **kw)
    o = oracle.estimate_pdf(4e-3, cfg, 0.0, 100.0, 10,
                            estimator=oracle.STMC if estimator == "stmc" else oracle.MLMC, **kw)
    say(f"pdf {estimator}: N={g['N']} L={g['L']} oracle N={o['N']} L={o['L']} "
        f"{g['wall_seconds'] * 1e3:.1f} ms")
    assert g["N"] == o["N"] and g["L"] == o["L"] and g["status"] == o["status"]
    for a, b in zip(g["estimate"], o["estimate"]):
        assert abs(a - b) <= 1e-11, (a, b)


def test_range_longer_than_a_chunk():
    cfg = W.neutral(500.0, "BAOAB", r=4, delta=100.0, M0=8)
    n = (1 << 22) + 12345
    whole = ld.pdf_level_sums(cfg, 0, 0, n, 0.0, 50.0, 20, precision="fp32")
    st = ld.estimate_pdf(1.0, cfg, 0.0, 50.0, 20, estimator="stmc", fixed_L=0, N_init=n,
                         precision="fp32", max_iter=1)
    assert st["N"] == [n]
    for i, x in enumerate(whole):
        assert x["n"] == n
        assert st["estimate"][i] == pytest.approx(x["sum_pf"] / x["n"], rel=1e-12, abs=1e-15)


def test_estimate_pdf_with_a_caller_workspace_or_its_own():
    """A caller's workspace (what the binding passes) and the library's own allocation
    (NULL through the C ABI) give the same estimate bit for bit; a workspace below
    mlmc_estimate_pdf_workspace() is refused with LD_ENOMEM."""
    import ctypes as C
    import torch
    cfg = W.neutral(200.0, "BAOAB", r=4, delta=100.0, M0=40)
    kw = dict(N_init=1000, L_max=6, precision="fp64")
    g = ld.estimate_pdf(1e-2, cfg, 0.0, 100.0, 10, **kw)
    lib = ld.load()
    o = ld.estimate_opts(cfg, eps_is_relative=False, **kw)      # d_workspace NULL
    r = ld.PdfResult()
    rc = lib.mlmc_estimate_pdf(1e-2, C.byref(ld.make_bins(0.0, 100.0, 10)), C.byref(ld.make_qoi(cfg)),
                               ld.INTEGRATORS["BAOAB"], C.byref(ld.make_profile(cfg)), C.byref(o),
                               ld.ESTIMATORS["mlmc"], C.byref(r))
    assert rc in (ld.LD_OK, ld.LD_WARN_NOT_CONVERGED)
    assert [int(r.N[l]) for l in range(r.L + 1)] == g["N"]
    assert list(r.estimate[:10]) == g["estimate"]
    need = int(lib.mlmc_estimate_pdf_workspace(10))
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(ld.LdError) as e:
        ld.estimate_pdf(1e-2, cfg, 0.0, 100.0, 10, workspace=small, **kw)
    assert e.value.status == ld.LD_ENOMEM
