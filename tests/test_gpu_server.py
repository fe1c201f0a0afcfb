"""GPU tests of the request server (continuous batching over the engine).

- Queries submitted while others run give bitwise the results they give alone
  (the served result equals a one-query engine run of the same query).
- Results do not depend on the order or timing of arrivals.
- The FIFO policy equals mlmc_estimate query by query (same driver, same draws).
- The admission queue bound answers LD_EBUSY; counters add up; clients on several
  threads can submit and wait at once.
"""
import sys
import threading
import time

import pytest

import oracle
import paper_1612_07717_amd as ld
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _queries(n, seed, eps_range=(3e-3, 2e-2)):
    qs = W.batched_estimators(n, seed=seed, eps_range=eps_range)
    return [ld.make_query(q["problem"], q["eps"], eps_is_relative=q["eps_is_relative"],
                          N_init=2000, L_max=10) for q in qs]


def test_served_results_equal_alone_results():
    qs = _queries(10, seed=21)
    alone = [ld.estimate_batch([q], precision="fp32")[0] for q in qs]
    with ld.Server(policy="batch", precision="fp32") as srv:
        tickets = []
        for i, q in enumerate(qs):
            tickets.append(srv.submit(q))
            if i % 3 == 2:
                time.sleep(0.002)          # let some queries start before others arrive
        served = [srv.wait(t, timeout=60.0) for t in tickets]
        st = srv.stats()
    assert all(s is not None for s in served)
    for a, (r, tm) in zip(alone, served):
        assert r["N"] == a["N"] and r["L"] == a["L"]
        assert r["estimate"] == a["estimate"]
        assert r["Yhat"] == a["Yhat"] and r["V"] == a["V"]
        assert tm["t_submit"] <= tm["t_admit"] <= tm["t_done"]
    say(f"served {st['completed']} queries in {st['iterations']} iterations, "
        f"max running {st['max_running']}")
    assert st["submitted"] == st["completed"] == len(qs)
    assert st["max_running"] >= 2           # the queries did share the device


def test_arrival_order_does_not_change_results():
    qs = _queries(8, seed=22)
    with ld.Server(policy="batch", precision="fp32") as srv:
        fwd = [srv.submit(q) for q in qs]
        a = [srv.wait(t, timeout=60.0)[0] for t in fwd]
    with ld.Server(policy="batch", precision="fp32", max_queries=3) as srv:
        rev = [srv.submit(q) for q in reversed(qs)]
        b = [srv.wait(t, timeout=60.0)[0] for t in rev][::-1]
    for x, y in zip(a, b):
        assert x["N"] == y["N"] and x["estimate"] == y["estimate"]


def test_fifo_policy_equals_mlmc_estimate_fp64():
    qs = W.batched_estimators(3, seed=23, eps_range=(1e-2, 2e-2))
    with ld.Server(policy="fifo", precision="fp64") as srv:
        tickets = [srv.submit(ld.make_query(q["problem"], q["eps"], N_init=2000, L_max=9,
                                            eps_is_relative=q["eps_is_relative"])) for q in qs]
        got = [srv.wait(t, timeout=120.0)[0] for t in tickets]
    for q, r in zip(qs, got):
        e = ld.estimate(q["eps"], q["problem"], precision="fp64",
                        eps_is_relative=q["eps_is_relative"], N_init=2000, L_max=9)
        say(f"fifo fp64 {q['problem']['integrator']}: {r['estimate']} vs {e['estimate']}")
        assert r["N"] == e["N"] and r["estimate"] == e["estimate"]


def test_queue_bound_and_threaded_clients():
    qs = _queries(12, seed=24)
    ref = {i: ld.estimate_batch([q], precision="fp32")[0] for i, q in enumerate(qs[:4])}
    with ld.Server(policy="batch", precision="fp32", max_queued=1, max_queries=1) as srv:
        # one slot and a one-deep queue: at most two queries are held
        t0 = srv.submit(qs[0])
        held = [t0]
        refused = 0
        for q in qs[1:4]:
            t = srv.submit(q)
            if t is None:
                refused += 1
            else:
                held.append(t)
        assert refused >= 1
        for t in held:
            assert srv.wait(t, timeout=60.0) is not None
    with ld.Server(policy="batch", precision="fp32") as srv:
        out = {}
        errors = []

        def client(idx):
            try:
                for i in idx:
                    t = srv.submit(qs[i])
                    out[i] = srv.wait(t, timeout=60.0)[0]
            except Exception as exc:   # noqa: BLE001 -- reported below
                errors.append(exc)

        th = [threading.Thread(target=client, args=(range(k, len(qs), 4),)) for k in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join(timeout=120.0)
        assert not errors and len(out) == len(qs)
        st = srv.stats()
        assert st["submitted"] == st["completed"] == len(qs) and st["queued"] == 0
    for i, a in ref.items():
        assert out[i]["estimate"] == a["estimate"] and out[i]["N"] == a["N"]


def test_cost_budget_stops_engine_and_driver_alike():
    """A query whose next batch would pass max_fine_steps stops with the warning status
    after the same batches in the engine, the server and mlmc_estimate."""
    c = W.neutral(300.0, "BAOAB")
    budget = 3e8
    d = ld.estimate(1e-4, c, precision="fp32", eps_is_relative=True, N_init=2000,
                    max_fine_steps=budget)
    q = ld.make_query(c, 1e-4, N_init=2000, max_fine_steps=budget)
    b = ld.estimate_batch([q], precision="fp32")[0]
    with ld.Server(policy="batch", precision="fp32") as srv:
        s = srv.wait(srv.submit(q), timeout=60.0)[0]
    say(f"budget stop: N={d['N']} steps={d['fine_steps']:.3g} status={d['status']}")
    assert d["rc"] == ld.LD_WARN_NOT_CONVERGED and d["status"] == 2
    assert d["fine_steps"] <= budget
    for r in (b, s):
        assert r["status"] == 2 and r["N"] == d["N"] and r["estimate"] == d["estimate"]
    free = ld.estimate(1e-4, c, precision="fp32", eps_is_relative=True, N_init=2000)
    assert free["fine_steps"] > budget and free["status"] == 1


@pytest.mark.parametrize("policy", ["batch", "fifo"])
def test_adaptive_queries_are_served(policy):
    """Adaptive symplectic Euler queries (Sec. 7) served beside uniform ones: each result
    equals mlmc_estimate's on the same query."""
    base = W.problem(integrator="SE", M0=40)
    cfgs = [dict(base, x_adapt=50.0), W.neutral(400.0, "GL"), dict(base, x_adapt=50.0, z0=90.0, seed=4)]
    with ld.Server(policy=policy, precision="fp32") as srv:
        tickets = [srv.submit(ld.make_query(c, 1e-2, N_init=2000, L_max=8)) for c in cfgs]
        got = [srv.wait(t, timeout=120.0)[0] for t in tickets]
    for c, r in zip(cfgs, got):
        e = ld.estimate(1e-2, c, precision="fp32", eps_is_relative=True, N_init=2000, L_max=8)
        assert r["N"] == e["N"] and r["estimate"] == e["estimate"]


def test_fp64_served_results_match_the_oracle_driver():
    """FP64 queries served together (continuous batching) against the oracle's own
    driver run on each query alone (Sec. 3.3, Sec. 6): the same samples per level and
    finest level, and estimates within 1e-11 relative."""
    cfgs = [(W.neutral(300.0, "GL", stream_id=3), 1e-2), (W.neutral(700.0, "BAOAB", stream_id=4), 1e-2),
            (W.problem(integrator="SE", stream_id=5), 2e-2),
            (W.neutral(450.0, "BAOAB", qoi="p_above", qa=400.0, r=4, delta=100.0, stream_id=6), 2e-2)]
    qs = [ld.make_query(c, e, N_init=3000, L_max=9) for c, e in cfgs]
    with ld.Server(policy="batch", precision="fp64") as srv:
        tickets = [srv.submit(q) for q in qs]
        served = [srv.wait(t, timeout=120.0) for t in tickets]
    for (c, e), got in zip(cfgs, served):
        assert got is not None
        r = got[0]
        o = oracle.estimate(e, c, eps_is_relative=True, N_init=3000, L_max=9)
        say(f"served fp64 {c['integrator']}: {r['estimate']} N={r['N']} oracle {o['estimate']} N={o['N']}")
        assert r["N"] == o["N"] and r["L"] == o["L"]
        assert r["estimate"] == pytest.approx(o["estimate"], rel=1e-11, abs=1e-13)

