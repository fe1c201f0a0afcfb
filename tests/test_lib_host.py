"""Host-side tests of the HIP library (no GPU needed).

- the library loads and exports every function include/ldmlmc.h declares;
- the ctypes structs of the binding match the C layout (sizes and offsets printed by a
  small C program compiled against the header);
- the library's planner (mlmc_plan) and the oracle's take the same decisions on the
  same inputs (the two are independent implementations of the algorithm);
- argument validation and the stability check reject bad input before any device use.
"""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1612_07717_amd as ld
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ldmlmc.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ld.LIB_PATH):
        from paper_1612_07717_amd import build
        build.build()
    return ld.load()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*\b([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("mlmc_", "ld_"))))


def test_exports_every_declared_function(lib):
    declared = _declared_functions()
    assert len(declared) >= 11
    assert sorted(declared) == sorted(ld.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", ld.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (\S+)", out))
    for name in declared:
        assert name in exported, name
        assert hasattr(lib, name)


def test_struct_layouts_match_header(tmp_path):
    structs = {"ld_profile": ld.Profile, "ld_qoi": ld.Qoi, "ld_release": ld.Release,
               "ld_problem": ld.Problem, "ld_level_sums": ld.LevelSums,
               "ld_level_range": ld.LevelRange, "ld_plan_in": ld.PlanIn,
               "ld_plan_out": ld.PlanOut, "ld_estimate_opts": ld.EstimateOpts,
               "ld_estimate_result": ld.EstimateResult, "ld_engine_opts": ld.EngineOpts,
               "ld_query": ld.Query, "ld_server_opts": ld.ServerOpts,
               "ld_request_times": ld.RequestTimes, "ld_server_stats": ld.ServerStats,
               "ld_bins": ld.Bins, "ld_pdf_plan_in": ld.PdfPlanIn, "ld_pdf_plan_out": ld.PdfPlanOut,
               "ld_pdf_result": ld.PdfResult}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ldmlmc.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'printf("{cname}.{field} %zu\\n", offsetof({cname}, {field}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True,
                                                              text=True, check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[f"{cname} size"]) == C.sizeof(py), cname
        for field, _ in py._fields_:
            assert int(got[f"{cname}.{field}"]) == getattr(py, field).offset, (cname, field)


def _random_plan_inputs(rng, n_cases):
    for _ in range(n_cases):
        L = int(rng.integers(0, 8))
        n = [int(rng.integers(2, 200000)) for _ in range(L + 1)]
        V = [float(10.0 ** rng.uniform(-5, 3)) * 4.0 ** -l for l in range(L + 1)]
        mean = [float(rng.normal(0, 3)) * 2.0 ** -l for l in range(L + 1)]
        s1 = [m * k for m, k in zip(mean, n)]
        s2 = [v * (k - 1) + k * m * m for v, k, m in zip(V, n, mean)]
        yield dict(L=L, n=n, sum1=s1, sum2=s2, M0=int(rng.choice([8, 40, 80])),
                   eps=float(10.0 ** rng.uniform(-3, 1)),
                   eps_is_relative=int(rng.integers(0, 2)), L_max=int(rng.integers(L, 12)),
                   fixed_L=int(rng.choice([-1, -1, L])), fixed_N=int(rng.integers(0, 10) == 0),
                   N_init=int(rng.choice([1000, 10000])), alpha=float(rng.choice([1.0, 2.0, 0.0])))


def test_planner_matches_oracle_planner(lib, orc):
    rng = np.random.default_rng(11)
    checked = 0
    for d in _random_plan_inputs(rng, 3000):
        a, b = ld.plan(d), orc.plan(d)
        assert a["status"] == b["status"] and a["L"] == b["L"], d
        assert a["dn"] == b["dn"], d
        for k in ("estimate", "eps_abs", "alpha", "bias_est", "stat_var"):
            assert a[k] == pytest.approx(b[k], rel=1e-12, abs=1e-300), (k, d)
        assert np.allclose(a["V"], b["V"], rtol=1e-12, atol=0)
        checked += 1
    assert checked == 3000


def test_planner_rejects_bad_input(lib):
    with pytest.raises(ld.LdError) as e:
        ld.plan(dict(L=-1, n=[], sum1=[], sum2=[], M0=8, eps=1.0))
    assert e.value.status == ld.LD_EINVAL
    with pytest.raises(ld.LdError):
        ld.plan(dict(L=1, n=[10, 10], sum1=[0, 0], sum2=[1, 1], M0=8, eps=0.0))


def _call_level_sums(lib, cfg, level=0, n=100, ws_bytes=None, integ=None):
    p = ld.make_problem(cfg)
    ws_bytes = ld.level_sums_workspace(n) if ws_bytes is None else ws_bytes
    fake = C.c_void_p(0x1000)   # never dereferenced: validation fails first
    return lib.mlmc_level_sums(C.byref(p), ld.INTEGRATORS[integ or cfg["integrator"]], 0, level, 0,
                               n, fake, fake, ws_bytes, None)


def test_validation_rejects_bad_problems_without_device(lib):
    good = W.neutral(300.0, "GL")
    bad = [dict(good, H=-1.0), dict(W.homogeneous(), H=1e-300, z0=0.0), dict(W.homogeneous(), H=1e31),
           dict(good, eps_reg=600.0), dict(good, eps_reg=0.0), dict(good, eps_reg=1e-4),
           dict(good, kappa_tau=0.0), dict(good, z0=1200.0), dict(good, T=0.0),
           dict(good, M0=0), dict(good, stream_id=1 << 24),
           dict(good, qoi="p_box", r=9, delta=100.0), dict(good, qoi="p_box", r=4, delta=0.0),
           dict(W.homogeneous(), tau=0.0), dict(W.homogeneous(), sigma_u=-1.0)]
    for cfg in bad:
        assert _call_level_sums(lib, cfg) == ld.LD_EINVAL, cfg
    assert _call_level_sums(lib, good, level=32) == ld.LD_EINVAL
    assert _call_level_sums(lib, dict(good, M0=1 << 20), level=12) == ld.LD_EINVAL   # M > 2^31


def test_symplectic_euler_stability_check(lib):
    """Sec. 3.1: SE needs lambda h < 2. At eps_reg = 10 m, M_0 = 8 (h = 125 s) violates it
    (lambda_max h = 6.45); M_0 = 40 does not. The coarse step of level l is 2 h_l."""
    assert _call_level_sums(lib, W.single_large("SE"), level=0) == ld.LD_EUNSTABLE
    assert _call_level_sums(lib, W.single_large("SE"), level=2) == ld.LD_EUNSTABLE   # 2h = 62.5 s
    assert _call_level_sums(lib, W.single_large("SE"), level=3, ws_bytes=0) == ld.LD_ENOMEM
    assert _call_level_sums(lib, W.single_large("BAOAB"), level=0, ws_bytes=0) == ld.LD_ENOMEM
    assert _call_level_sums(lib, W.neutral(500.0, "SE"), level=0, ws_bytes=0) == ld.LD_ENOMEM
    # homogeneous c1: lambda h_0 = 1.25 < 2
    assert _call_level_sums(lib, W.homogeneous(), level=0, ws_bytes=0) == ld.LD_ENOMEM


def test_estimate_argument_errors(lib):
    with pytest.raises(ld.LdError) as e:
        ld.estimate(0.0, W.neutral(300.0, "GL"))
    assert e.value.status == ld.LD_EINVAL
    with pytest.raises(ld.LdError) as e:
        ld.estimate(1.0, W.single_large("SE"))
    assert e.value.status == ld.LD_EUNSTABLE
    with pytest.raises(ld.LdError) as e:
        ld.estimate(1.0, W.neutral(300.0, "GL"), L_min=5, L_max=3)
    assert e.value.status == ld.LD_EINVAL


def test_strerror_covers_all_codes(lib):
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6, -7):
        assert lib.ld_strerror(code).decode() != "unknown status"
    assert lib.ld_strerror(-99).decode() == "unknown status"


def test_batch_validates_queries_before_device_use(lib):
    bad = ld.make_query(W.neutral(300.0, "GL", H=-5.0), 1e-2)
    good = ld.make_query(W.neutral(300.0, "GL"), 1e-2)
    arr = (ld.Query * 2)(good, bad)
    res = (ld.EstimateResult * 2)()
    assert lib.mlmc_estimate_batch(arr, 2, None, res) == ld.LD_EINVAL
    unstable = ld.make_query(W.single_large("SE"), 1e-2)
    arr = (ld.Query * 1)(unstable)
    assert lib.mlmc_estimate_batch(arr, 1, None, res) == ld.LD_EUNSTABLE
    assert lib.mlmc_estimate_batch(arr, 0, None, res) == ld.LD_EINVAL
    assert lib.ld_engine_run(None, arr, 1, res) == ld.LD_EINVAL


def test_server_rejects_bad_arguments_without_device(lib):
    """Server entry points check their arguments before any device use; creating a
    server with no GPU present fails with a status, not a crash."""
    h = C.c_void_p()
    bad = ld.ServerOpts()
    lib.ld_server_default_opts(C.byref(bad))
    bad.policy = 7
    assert lib.ld_server_create(C.byref(bad), C.byref(h)) == ld.LD_EINVAL
    bad.policy = 0
    bad.max_queued = -1
    assert lib.ld_server_create(C.byref(bad), C.byref(h)) == ld.LD_EINVAL
    t = C.c_int64()
    q = ld.make_query(W.neutral(300.0, "GL"), 1e-2)
    assert lib.ld_server_submit(None, C.byref(q), C.byref(t)) == ld.LD_EINVAL
    r = ld.EstimateResult()
    assert lib.ld_server_wait(None, 0, 0.0, C.byref(r), None) == ld.LD_EINVAL
    a, b = lib.ld_server_clock(), lib.ld_server_clock()
    assert b >= a


def test_negative_cost_budget_is_rejected(lib):
    q = ld.make_query(W.neutral(300.0, "GL"), 1e-2, max_fine_steps=-1.0)
    res = (ld.EstimateResult * 1)()
    assert lib.mlmc_estimate_batch((ld.Query * 1)(q), 1, None, res) == ld.LD_EINVAL
    with pytest.raises(ld.LdError) as e:
        ld.estimate(1e-2, W.neutral(300.0, "GL"), max_fine_steps=-1.0)
    assert e.value.status == ld.LD_EINVAL


def _random_pdf_inputs(rng, n_cases):
    for _ in range(n_cases):
        L = int(rng.integers(0, 7))
        k = int(rng.integers(1, 25))
        n = [int(rng.integers(2, 200000)) for _ in range(L + 1)]
        s1 = [[0.0] * k for _ in range(L + 1)]
        s2 = [[0.0] * k for _ in range(L + 1)]
        for l in range(L + 1):
            for i in range(k):
                mean = float(rng.normal(0, 0.05)) * 2.0 ** -l
                var = float(10.0 ** rng.uniform(-6, -1)) * 4.0 ** -l
                s1[l][i] = mean * n[l]
                s2[l][i] = var * (n[l] - 1) + n[l] * mean * mean
        yield dict(L=L, n_bins=k, n=n, sum1=s1, sum2=s2, M0=int(rng.choice([8, 40, 80])),
                   eps=float(10.0 ** rng.uniform(-4, -1)), L_max=int(rng.integers(L, 12)),
                   fixed_L=int(rng.choice([-1, -1, L])), N_init=int(rng.choice([1000, 10000])),
                   alpha=float(rng.choice([1.0, 2.0, 0.0])))


def test_pdf_planner_matches_oracle_planner(lib, orc):
    rng = np.random.default_rng(12)
    for d in _random_pdf_inputs(rng, 600):
        a, b = ld.pdf_plan(d), orc.pdf_plan(d)
        assert (a["status"], a["L"], a["dn"]) == (b["status"], b["L"], b["dn"]), d["L"]
        for key in ("bias_est", "stat_var", "alpha"):
            assert a[key] == pytest.approx(b[key], rel=1e-12, abs=1e-300), key
        assert np.allclose(a["estimate"], b["estimate"], rtol=1e-12, atol=1e-300)
        assert np.allclose(a["V"], b["V"], rtol=1e-12, atol=0)


def test_pdf_arguments_rejected_without_device(lib):
    cfg = W.neutral(300.0, "GL", r=4, delta=100.0)
    p = ld.make_problem(cfg)
    fake = C.c_void_p(0x1000)   # never dereferenced: validation fails first
    for bins in (ld.make_bins(0.0, 50.0, 0), ld.make_bins(0.0, 50.0, 65), ld.make_bins(0.0, 0.0, 20),
                 ld.make_bins(float("nan"), 50.0, 20)):
        assert lib.mlmc_pdf_level_sums(C.byref(p), 1, 0, 0, 0, 100, C.byref(bins), fake, fake,
                                       1 << 30, None) == ld.LD_EINVAL
    bad_r = ld.make_problem(dict(cfg, r=9))
    assert lib.mlmc_pdf_level_sums(C.byref(bad_r), 1, 0, 0, 0, 100, C.byref(ld.make_bins(0.0, 50.0, 20)),
                                   fake, fake, 1 << 30, None) == ld.LD_EINVAL
    good = ld.make_bins(0.0, 50.0, 20)
    assert lib.mlmc_pdf_level_sums(C.byref(p), 1, 0, 0, 0, 100, C.byref(good), fake, fake, 0,
                                   None) == ld.LD_ENOMEM
    assert lib.mlmc_pdf_level_sums_workspace(1000, 0) == 0
    assert lib.mlmc_pdf_level_sums_workspace(1000, 20) >= 16 * 1000
    assert lib.mlmc_estimate_pdf_workspace(0) == 0 and lib.mlmc_estimate_pdf_workspace(65) == 0
    # the estimate's workspace holds a whole dump chunk (16 B per sample) and the sums of
    # every bin, and grows with the bin count
    assert lib.mlmc_estimate_pdf_workspace(64) > lib.mlmc_estimate_pdf_workspace(1) >= 16 << 22
    res = ld.PdfResult()
    q, prof = ld.make_qoi(cfg), ld.make_profile(cfg)
    o = ld.estimate_opts(cfg)
    assert lib.mlmc_estimate_pdf(1e-3, C.byref(good), C.byref(q), 1, C.byref(prof), C.byref(o),
                                 1, C.byref(res)) == ld.LD_EINVAL       # StMC needs fixed_L
    o_rel = ld.estimate_opts(cfg, eps_is_relative=True)
    assert lib.mlmc_estimate_pdf(1e-3, C.byref(good), C.byref(q), 1, C.byref(prof), C.byref(o_rel),
                                 0, C.byref(res)) == ld.LD_EINVAL       # absolute eps only
    assert lib.mlmc_estimate_pdf(1e-3, C.byref(good), C.byref(q), 1, C.byref(prof), C.byref(o),
                                 5, C.byref(res)) == ld.LD_EINVAL       # unknown estimator
    o_small = ld.estimate_opts(cfg)
    o_small.d_workspace, o_small.workspace_bytes = fake.value, 4096    # refused before any use
    assert lib.mlmc_estimate_pdf(1e-3, C.byref(good), C.byref(q), 1, C.byref(prof), C.byref(o_small),
                                 0, C.byref(res)) == ld.LD_ENOMEM


def test_adaptive_steps_validation_and_stability(lib):
    """x_adapt > 0 selects the adaptive symplectic Euler of Sec. 7: SE only, the
    stability condition uses lambda(x_adapt) (dt_0 = T/8 becomes stable with x_adapt =
    50 m); the engine takes adaptive queries under the same limits."""
    se8 = W.single_large("SE")                                   # M0 = 8: lambda_max h_0 = 6.45
    assert _call_level_sums(lib, se8, level=0) == ld.LD_EUNSTABLE
    ada = dict(se8, x_adapt=50.0)                                # lambda(50 m) h_0 = 1.25
    assert _call_level_sums(lib, ada, level=0, ws_bytes=0) == ld.LD_ENOMEM
    assert _call_level_sums(lib, dict(ada, integrator="GL"), level=0) == ld.LD_EINVAL
    assert _call_level_sums(lib, dict(ada, x_adapt=-1.0), level=0) == ld.LD_EINVAL
    assert _call_level_sums(lib, dict(ada, x_adapt=2000.0), level=0) == ld.LD_EINVAL
    assert _call_level_sums(lib, dict(ada, x_adapt=900.0), level=0) == ld.LD_EINVAL   # > 64x shorter steps
    assert _call_level_sums(lib, dict(ada, M0=1 << 20), level=7) == ld.LD_EINVAL      # M > 2^26
    q = ld.make_query(ada, 1e-2, L_max=24)                       # M0 2^L_max = 2^27 > 2^26
    res = (ld.EstimateResult * 1)()
    assert lib.mlmc_estimate_batch((ld.Query * 1)(q), 1, None, res) == ld.LD_EINVAL
    q = ld.make_query(dict(ada, integrator="GL"), 1e-2)          # adaptive steps: SE only
    assert lib.mlmc_estimate_batch((ld.Query * 1)(q), 1, None, res) == ld.LD_EINVAL


def test_estimate_without_a_device_reports_it(lib):
    """Valid arguments on a machine without a GPU: LD_ENODEVICE, no crash, no fallback."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    cfg = W.neutral(500.0, "BAOAB")
    o = ld.estimate_opts(cfg, eps_is_relative=True)
    r = ld.EstimateResult()
    q, prof = ld.make_qoi(cfg), ld.make_profile(cfg)
    rc = lib.mlmc_estimate(1e-2, C.byref(q), ld.INTEGRATORS["BAOAB"], C.byref(prof), C.byref(o), C.byref(r))
    assert rc == ld.LD_ENODEVICE


def test_device_code_flags_fix_the_rounding():
    """PIPE and STREAM blocks inline the same step and must round alike, so an FMA comes
    only from a * b + c within one expression (-ffp-contract=on, not HIP's 'fast');
    no fast-math (the compensated sums need IEEE semantics); packed FP32 stays off."""
    from paper_1612_07717_amd import build
    f = build.HIPCC_FLAGS
    assert "-ffp-contract=on" in f and "-fno-fast-math" in f
    assert not any(x.startswith("-ffast-math") or x == "-ffp-contract=fast" for x in f)
    i = f.index("-packed-fp32-ops")
    assert f[i - 1] == "-Xclang" and f[i - 2] == "-target-feature" and f[i - 3] == "-Xclang"


def test_noalloc_level_sums_validates_before_device_use(lib):
    """mlmc_level_sums_noalloc takes no workspace; its arguments are checked as
    mlmc_level_sums checks them, before any device call."""
    good = W.neutral(300.0, "GL")
    fake = C.c_void_p(0x1000)   # never dereferenced: validation fails first
    for cfg, level in ((dict(good, H=-1.0), 0), (dict(good, M0=0), 0), (good, 32),
                       (dict(good, M0=1 << 20), 12)):
        p = ld.make_problem(cfg)
        assert lib.mlmc_level_sums_noalloc(C.byref(p), 1, 0, level, 0, 100, fake, None) == ld.LD_EINVAL
    p = ld.make_problem(good)
    assert lib.mlmc_level_sums_noalloc(C.byref(p), 7, 0, 0, 0, 100, fake, None) == ld.LD_EINVAL
    assert lib.mlmc_level_sums_noalloc(C.byref(p), 1, 0, 0, 0, 100, None, None) == ld.LD_EINVAL
