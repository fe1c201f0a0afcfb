"""GPU tests of the multi-estimator engine (persistent tile kernel, graph replay,
continuous batching).

- A batch of queries gives exactly the estimates of separate mlmc_estimate calls
  (same tiling rule per range, same compensated merges, same planner decisions).
- A query's result is bitwise the same alone and mixed with other queries.
- FP64 engine estimates equal the oracle's adaptive estimates (same N_l).
- Admission under a small slot budget, release and re-admission; graph replay
  equals direct launches.
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


def _mixed_configs(n, seed=3):
    """Neutral-layer queries of the batched workload, with tolerances loose enough for
    a quick test."""
    qs = W.batched_estimators(n, seed=seed, eps_range=(5e-3, 2e-2))
    return [(q["problem"], q["eps"], q["eps_is_relative"]) for q in qs]


def _query(c, e, rel, **kw):
    return ld.make_query(c, e, eps_is_relative=rel, **kw)


def test_batch_equals_single_estimates():
    cfgs = _mixed_configs(6)
    qs = [_query(c, e, rel, N_init=2000, L_max=10) for c, e, rel in cfgs]
    batch = ld.estimate_batch(qs, precision="fp32")
    for (c, e, rel), b in zip(cfgs, batch):
        s = ld.estimate(e, c, precision="fp32", eps_is_relative=rel, N_init=2000, L_max=10)
        say(f"batch {c['integrator']} z0={c['z0']:.0f} {c['qoi']}: {b['estimate']:.6f} N={b['N']}")
        assert b["N"] == s["N"] and b["L"] == s["L"]
        assert b["estimate"] == s["estimate"]
        assert b["status"] == s["status"] == 1
    assert not all(rel for _, _, rel in cfgs) and any(rel for _, _, rel in cfgs)


def test_engine_run_equals_batch_and_keeps_the_engine():
    """ld_engine_run on a live engine gives mlmc_estimate_batch's results bit for bit, twice
    in a row on the same engine (each query's sums start from zero when it is admitted)."""
    cfgs = _mixed_configs(9, seed=17)
    qs = [_query(c, e, rel, N_init=1000, L_max=9) for c, e, rel in cfgs]
    ref = ld.estimate_batch(qs, precision="fp32", max_queries=4)
    with ld.Engine(precision="fp32", max_queries=4) as eng:   # fewer slots than queries
        for rep in range(2):
            got = eng.run(qs)
            for r, g in zip(ref, got):
                assert g["N"] == r["N"] and g["estimate"] == r["estimate"], rep
        assert eng.stats()["iterations"] > 0


def test_alone_equals_mixed_bitwise():
    cfgs = _mixed_configs(12, seed=5)
    q0 = _query(*cfgs[0], N_init=2000, L_max=10)
    alone = ld.estimate_batch([q0], precision="fp32")[0]
    mixed = ld.estimate_batch([_query(c, e, rel, N_init=2000, L_max=10) for c, e, rel in cfgs],
                              precision="fp32")[0]
    assert alone["N"] == mixed["N"]
    assert alone["estimate"] == mixed["estimate"]
    assert alone["Yhat"] == mixed["Yhat"] and alone["V"] == mixed["V"]


def test_fp64_engine_matches_oracle_driver():
    cfgs = [(W.neutral(300.0, "GL"), 1e-2), (W.neutral(700.0, "BAOAB"), 1e-2),
            (W.problem(integrator="SE"), 2e-2),
            (W.neutral(450.0, "BAOAB", qoi="p_above", qa=400.0, r=4, delta=100.0), 2e-2)]
    qs = [ld.make_query(c, e, N_init=3000, L_max=9) for c, e in cfgs]
    res = ld.estimate_batch(qs, precision="fp64")
    for (c, e), r in zip(cfgs, res):
        o = oracle.estimate(e, c, eps_is_relative=True, N_init=3000, L_max=9)
        say(f"fp64 engine {c['integrator']}: {r['estimate']} N={r['N']} oracle {o['estimate']} N={o['N']}")
        assert r["N"] == o["N"] and r["L"] == o["L"]
        assert r["estimate"] == pytest.approx(o["estimate"], rel=1e-11, abs=1e-13)


def test_admission_release_and_graph_equivalence():
    cfgs = _mixed_configs(7, seed=9)
    qs = [_query(c, e, rel, N_init=2000, L_max=10) for c, e, rel in cfgs]
    ref = ld.estimate_batch(qs, precision="fp32", use_graph=False)
    with ld.Engine(precision="fp32", max_queries=3, use_graph=True) as eng:   # graph-captured iterations
        handles = [eng.submit(q) for q in qs[:3]]
        assert all(h is not None for h in handles)
        assert eng.submit(qs[3]) is None                 # LD_EBUSY: no slot
        pending = list(range(3, len(qs)))
        owner = {h: i for i, h in enumerate(handles)}
        results = {}
        steps = 0
        while len(results) < len(qs):
            eng.step()
            steps += 1
            for h, i in list(owner.items()):
                r = eng.result(h)
                if r is not None:
                    results[i] = r
                    eng.release(h)
                    del owner[h]
            while pending:
                h = eng.submit(qs[pending[0]])
                if h is None:
                    break
                owner[h] = pending.pop(0)
            assert steps < 500
        st = eng.stats()
        assert st["iterations"] == steps and st["device_seconds"] > 0
    for i, r in results.items():
        assert r["N"] == ref[i]["N"] and r["estimate"] == ref[i]["estimate"]


def test_autotuner_returns_a_valid_configuration():
    cfgs = _mixed_configs(4, seed=13)
    qs = [_query(c, e, rel, N_init=1000, L_max=8) for c, e, rel in cfgs]
    best, t = ld.autotune(qs, reps=1, precision="fp32")
    d = ld.opts_dict(best)
    say(f"autotune best {d} in {t * 1e3:.2f} ms")
    assert d["blocks_per_cu"] in (2, 4, 6, 8, 12, 16) and t > 0
    res = ld.estimate_batch(qs, opts=best)
    assert all(r["status"] == 1 for r in res)


def test_mixed_profiles_batch_equals_single():
    """Queries of both turbulence profiles in one engine (both persistent kernels run),
    and a batch of homogeneous queries only (the neutral kernel is left out)."""
    cfgs = [(W.homogeneous(), 2e-2), (W.neutral(400.0, "GL"), 1e-2),
            (W.homogeneous(z0=300.0, integrator="BAOAB"), 2e-2), (W.neutral(650.0, "BAOAB"), 1e-2)]
    qs = [ld.make_query(c, e, N_init=2000, L_max=8) for c, e in cfgs]
    mixed = ld.estimate_batch(qs, precision="fp32")
    homog = ld.estimate_batch([qs[0], qs[2]], precision="fp32")
    for (c, e), m in zip(cfgs, mixed):
        s = ld.estimate(e, c, precision="fp32", eps_is_relative=True, N_init=2000, L_max=8)
        say(f"{c['profile']} {c['integrator']}: {m['estimate']:.6f} N={m['N']}")
        assert m["N"] == s["N"] and m["estimate"] == s["estimate"]
    assert homog[0]["estimate"] == mixed[0]["estimate"] and homog[1]["estimate"] == mixed[2]["estimate"]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_adaptive_queries_equal_single_estimates(prec):
    """Adaptive symplectic Euler queries (Sec. 7) run in the engine's third queue, mixed
    with uniform queries of both profiles; each equals its mlmc_estimate bit for bit."""
    base = W.problem(integrator="SE", M0=40)
    cfgs = [(dict(base, x_adapt=50.0), 5e-3, True),
            (dict(base, x_adapt=50.0, z0=120.0, seed=9), 1e-2, True),
            (W.neutral(300.0, "BAOAB"), 5e-3, True),
            (W.homogeneous(x_adapt=50.0), 1e-2, True)]
    qs = [_query(c, e, rel, N_init=2000, L_max=8) for c, e, rel in cfgs]
    batch = ld.estimate_batch(qs, precision=prec)
    for (c, e, rel), b in zip(cfgs, batch):
        s = ld.estimate(e, c, precision=prec, eps_is_relative=rel, N_init=2000, L_max=8)
        say(f"engine {prec} {c['integrator']} x_adapt={c.get('x_adapt', 0)}: {b['estimate']:.6f} N={b['N']}")
        assert b["N"] == s["N"] and b["L"] == s["L"]
        assert b["estimate"] == s["estimate"]
        assert b["status"] == s["status"] == 1


def test_adaptive_query_with_64_bit_ticks_equals_single_estimate():
    """Levels 0..7 at M_0 = 40: level 7 (5120 steps) needs 64-bit tick counters, the
    persistent kernel's other adaptive branch; the engine equals mlmc_estimate."""
    cfg = W.problem(integrator="SE", M0=40, x_adapt=50.0)
    q = _query(cfg, 1e-2, True, N_init=300, fixed_L=7)
    b = ld.estimate_batch([q], precision="fp32")[0]
    s = ld.estimate(1e-2, cfg, precision="fp32", eps_is_relative=True, N_init=300, fixed_L=7)
    assert b["L"] == s["L"] == 7
    assert b["N"] == s["N"] and b["estimate"] == s["estimate"]
