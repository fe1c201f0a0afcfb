"""Benchmark: coupled particle-steps/s of the MLMC dispersion hot path on one MI355X.

One step = one full adaptive MLMC estimate (all levels, the driver's iterations, the
level kernels and the FP64 planning) of the large single-estimate workload: neutral
boundary layer, BAOAB, release at 500 m with Gaussian w0, T = 1000 s, dt_0 = T/8,
levels 0..12, relative eps 1e-4, E[Z(T)], FP32 paths with FP64 compensated sums.
The line also carries a short serving run (Poisson arrivals, continuous batching,
p50/p99 latency, FP32 against plain one-at-a-time FP64).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32|fp64]
    python bench.py --workload batched      # 64 estimators in one engine
    python bench.py --workload serving --rate 100 --duration 60

Prints one JSON line. The CPU baseline times the oracle on a bounded sample of the
same workload on this host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import struct
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

# Peak figures of one MI355X (public): 256 CUs at 2.4 GHz. FP32 vector 157.3 TFLOP/s
# counts packed FMA (two FP32 FMAs per lane per clock), which this build never emits;
# without packing the FP32 vector peak is that of FP64, 78.6 TFLOP/s (one FMA per lane
# per clock: 256 CUs x 64 lanes x 2 FLOP x 2.4 GHz).
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}
PEAK_TFLOPS_UNPACKED = {"fp32": 78.6, "fp64": 78.6}

# Operations the method performs per coupled fine step (one fine step, half a coarse
# step, half a coupling, one normal and half a Philox block), counted from the
# equations: floating-point ALU operations (add, multiply, multiply-add, compare,
# min/max, select; each counts one) plus elementary functions (square root,
# reciprocal, exp/expm1, log, sine/cosine; one each), and apart from them the integer
# operations of the generator. BAOAB: 70 + 13 and 25; symplectic Euler and geometric
# Langevin: 50 + 10 and 25. Breakdown in DESIGN.md ("Algorithmic work per coupled step").
FP_OPS_PER_COUPLED_STEP = {"BAOAB": 83.0, "GL": 60.0, "SE": 60.0}
INT_OPS_PER_COUPLED_STEP = 25.0

INTEGRATOR_INDEX = {"SE": 0, "GL": 1, "BAOAB": 2}


def dominant_kernel(precision: str = "fp32", integrator: str = "BAOAB") -> str:
    """Symbol of the level kernel of the neutral profile that runs the estimate."""
    t = "f" if precision == "fp32" else "d"
    return f"_ZN3ldm12level_kernelI{t}Li{INTEGRATOR_INDEX[integrator]}ELi1EEEvNS_5KArgsEP13ld_level_sumsPd"


DOMINANT_KERNEL = dominant_kernel()


def _elf_sections(blob: bytes, base: int = 0):
    """(name, addr, offset, size) of every section of the ELF64 image at blob[base:]."""
    shoff = struct.unpack_from("<Q", blob, base + 0x28)[0]
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", blob, base + 0x3A)
    raw = [struct.unpack_from("<IIQQQQ", blob, base + shoff + i * shentsize) for i in range(shnum)]
    names_off = base + raw[shstrndx][4]

    def name(o):
        end = blob.index(b"\0", names_off + o)
        return blob[names_off + o:end].decode()
    return [(name(r[0]), r[3], base + r[4], r[5]) for r in raw]


def kernel_hash(symbol: str = DOMINANT_KERNEL) -> str:
    """sha256 (16 hex digits) of one kernel's gfx950 machine code in the built library:
    the bytes of its symbol in the code object of the library's offload bundle. Counter
    summaries committed under profiles/ carry it, and go stale exactly when that kernel's
    code changes. 'missing' if the library or the kernel cannot be read."""
    try:
        with open(os.path.join(ROOT, "paper_1612_07717_amd", "libldmlmc.so"), "rb") as f:
            lib = f.read()
        fat = next(s for s in _elf_sections(lib) if s[0] == ".hip_fatbin")
        b = fat[2]
        if lib[b:b + 24] != b"__CLANG_OFFLOAD_BUNDLE__":
            return "missing"
        n = struct.unpack_from("<Q", lib, b + 24)[0]
        pos, co = b + 32, None
        for _ in range(n):
            off, size, id_len = struct.unpack_from("<QQQ", lib, pos)
            ident = lib[pos + 24:pos + 24 + id_len]
            pos += 24 + id_len
            if b"gfx950" in ident:
                co = (b + off, size)
        if co is None:
            return "missing"
        secs = {s[0]: s for s in _elf_sections(lib, co[0])}
        sym, strs, text = secs[".symtab"], secs[".strtab"], secs[".text"]
        for i in range(sym[3] // 24):
            st_name, _, _, _, st_value, st_size = struct.unpack_from("<IBBHQQ", lib, sym[2] + 24 * i)
            end = lib.index(b"\0", strs[2] + st_name)
            if lib[strs[2] + st_name:end].decode() == symbol:
                start = text[2] + (st_value - text[1])
                return hashlib.sha256(lib[start:start + st_size]).hexdigest()[:16]
    except (OSError, StopIteration, KeyError, struct.error, ValueError):
        pass
    return "missing"


def hbm_traffic(precision: str, integrator: str = "BAOAB"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None when
    the summary is missing or the kernel's machine code changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"level_kernel_{precision}_single_large_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except OSError:
        return None
    if d.get("kernel_hash") != kernel_hash(dominant_kernel(precision, integrator)):
        return None
    return d.get("bytes_per_launch")


def valu_issue(precision: str, integrator: str = "BAOAB"):
    """Measured VALU issue utilisation of the dominant kernel's launches (committed
    rocprofv3 counter summary), or None when missing or taken on other machine code."""
    path = os.path.join(ROOT, "profiles", f"level_kernel_{precision}_single_large_valu.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except OSError:
        return None
    if d.get("kernel_hash") != kernel_hash(dominant_kernel(precision, integrator)):
        return None
    return {f"{r['blocks']}_blocks": round(r["issue_frac"], 3) for r in d["launches"] if r.get("issue_frac")}


def roofline(precision: str, integrator: str, fine_steps: float, kernel_seconds: float,
             launches: int) -> dict:
    """ALU roofline of the level kernel over the timed estimates: the algorithmic
    floating-point operations (FP_OPS_PER_COUPLED_STEP per coupled fine step) over the
    kernel time measured with HIP events on the launch streams (summed over launches),
    against the published vector peak and the peak without packed FP32."""
    fp = FP_OPS_PER_COUPLED_STEP[integrator]
    achieved = fp * fine_steps / kernel_seconds / 1e12
    peak, unpacked = PEAK_TFLOPS[precision], PEAK_TFLOPS_UNPACKED[precision]
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": hbm_traffic(precision, integrator),
            "kernel": f"level_kernel<{'float' if precision == 'fp32' else 'double'}, {integrator}, neutral>",
            "fp_ops_per_coupled_step": fp, "int_ops_per_coupled_step": INT_OPS_PER_COUPLED_STEP,
            "int_tops": INT_OPS_PER_COUPLED_STEP * fine_steps / kernel_seconds / 1e12,
            "peak_unpacked": unpacked, "frac_unpacked": achieved / unpacked,
            "coupled_steps": fine_steps, "launches": launches,
            "avg_launch_ms": 1e3 * kernel_seconds / launches,
            "valu_issue_util": valu_issue(precision, integrator)}


def _cpu_model() -> str:
    """The host CPU as /proc/cpuinfo names it: model name, family/model/stepping and
    the clock of the first processor entry."""
    fields = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not line.strip():
                    break
                k, _, v = line.partition(":")
                fields[k.strip()] = v.strip()
    except OSError:
        return "unknown"
    return (f"{fields.get('model name', 'unknown')} (family {fields.get('cpu family', '?')}, "
            f"model {fields.get('model', '?')}, stepping {fields.get('stepping', '?')}, "
            f"{fields.get('cpu MHz', '?')} MHz)")


def cpu_baseline(cfg, eps, fixed_L, N_init, one_core_steps=1.2e7):
    """The oracle as it stands on this host: its own MLMC driver (plain schedule) on the
    same estimate, giving time-to-eps and coupled particle-steps/s on all of the oracle's
    threads; then a bounded sample of the same levels on one thread (the figure to set
    beside the paper's single-core timings)."""
    import oracle

    threads = oracle.num_threads()
    t0 = time.perf_counter()
    r = oracle.estimate(eps, cfg, fixed_L=fixed_L, N_init=N_init, eps_is_relative=True)
    dt = time.perf_counter() - t0
    N = r["N"]
    total = sum(n * (cfg["M0"] << l) for l, n in enumerate(N))
    f1 = min(1.0, one_core_steps / total)
    counts = [max(64, int(n * f1)) for n in N]
    steps1 = sum(n * (cfg["M0"] << l) for l, n in enumerate(counts))
    oracle.set_num_threads(1)
    try:
        t1 = time.perf_counter()
        for l, n in enumerate(counts):
            oracle.level_sums(cfg, l, 0, n)
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_num_threads(threads)
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"value": r["fine_steps"] / dt, "unit": "coupled particle-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"the whole estimate by the oracle's own driver (plain schedule, FP64): "
                      f"N_l = {N}, {r['fine_steps']:.3g} coupled fine steps, {dt:.1f} s",
            "time_to_eps_s": dt, "estimate_m": r["estimate"], "rmse_est_m": r["rmse_est"],
            "one_core": {"value": steps1 / dt1, "sample": f"each level's N_l scaled by {f1:.3g}, "
                                                          f"{steps1:.3g} coupled fine steps, {dt1:.1f} s"},
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(), "cpus_usable": affinity}


def _pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if xs else None


# Per-query cost budget of the serving runs (coupled fine steps): about 25 ms of the
# FP32 path at full device rate and 10x the costliest well-posed query of the mix.
SERVE_MAX_FINE_STEPS = 1e10


def serve_trace(ld, arrivals, policy, precision, n_init, max_seconds=None, drain_seconds=120.0,
                **engine_kw):
    """Replays an arrival trace against a server in real time: each query is submitted
    at its arrival time, latency = completion - scheduled arrival. With max_seconds,
    submission stops at that time of the trace. Queries not done drain_seconds after
    the last submission are reported as unfinished (an overloaded server is not waited
    on for ever); their latency counts as the time they had waited by then."""
    queries = [ld.make_query(a["problem"], a["eps"], eps_is_relative=a["eps_is_relative"],
                             N_init=n_init, max_fine_steps=SERVE_MAX_FINE_STEPS) for a in arrivals]
    with ld.Server(policy=policy, precision=precision, **engine_kw) as srv:
        t0 = ld.clock() + 0.05
        sent = []
        next_note = t0 + 10.0
        for a, q in zip(arrivals, queries):
            if max_seconds is not None and a["arrival"] > max_seconds:
                break
            target = t0 + a["arrival"]
            while True:
                now = ld.clock()
                dt = target - now
                if dt <= 0:
                    break
                time.sleep(min(dt, 0.002) if dt > 0.0005 else 0)
            sent.append((srv.submit(q), target))
            if ld.clock() > next_note:
                st = srv.stats()
                print(json.dumps({"progress": f"{policy}/{precision} submitting",
                                  "submitted": st["submitted"], "completed": st["completed"],
                                  "running": st["running"], "queued": st["queued"]}),
                      file=sys.stderr, flush=True)
                next_note += 10.0
        deadline = ld.clock() + drain_seconds
        lat, queue_wait, steps, statuses = [], [], 0.0, {}
        unfinished = 0
        t_last = t0
        for ticket, target in sent:
            got = None
            while got is None:
                left = deadline - ld.clock()
                if left <= 0:
                    break
                got = srv.wait(ticket, timeout=min(left, 10.0))
                if got is None:
                    st = srv.stats()
                    print(json.dumps({"progress": f"{policy}/{precision} draining",
                                      "completed": st["completed"], "of": len(sent),
                                      "running": st["running"], "queued": st["queued"]}),
                          file=sys.stderr, flush=True)
            if got is None:
                unfinished += 1
                lat.append(ld.clock() - target)
                continue
            r, tm = got
            lat.append(tm["t_done"] - target)
            queue_wait.append(tm["t_admit"] - tm["t_submit"])
            steps += r["fine_steps"]
            statuses[r["status"]] = statuses.get(r["status"], 0) + 1
            t_last = max(t_last, tm["t_done"])
        st = srv.stats()
    span = (ld.clock() if unfinished else t_last) - t0
    return {"policy": policy, "precision": precision, "queries": len(sent),
            "unfinished": unfinished,
            "p50_ms": 1e3 * _pct(lat, 50), "p99_ms": 1e3 * _pct(lat, 99),
            "mean_ms": 1e3 * sum(lat) / len(lat), "max_ms": 1e3 * max(lat),
            "admission_wait_p99_ms": 1e3 * _pct(queue_wait, 99) if queue_wait else None,
            "queries_per_s": (len(sent) - unfinished) / span, "span_s": span,
            "coupled_steps_per_s": steps / span, "iterations": st["iterations"],
            "max_running": st["max_running"], "max_queued": st["max_queued"],
            "device_busy_frac": st["device_seconds"] / span,
            "status_counts": {str(k): v for k, v in sorted(statuses.items())}}


def serving_report(ld, rate, duration, seed, n_init, fifo_seconds=None, precisions=("fp32", "fp64"),
                   **engine_kw):
    arrivals = W.poisson_arrivals(rate, duration, seed=seed)
    out = {"rate_qps": rate, "duration_s": duration, "arrivals": len(arrivals),
           "eps_range": [3e-4, 1e-2], "N_init": n_init, "max_fine_steps": SERVE_MAX_FINE_STEPS,
           "runs": []}
    for prec in precisions:
        out["runs"].append(serve_trace(ld, arrivals, "batch", prec, n_init, **engine_kw))
        print(json.dumps({"progress": "serving", **out["runs"][-1]}), file=sys.stderr, flush=True)
    out["runs"].append(serve_trace(ld, arrivals, "fifo", "fp64", n_init, max_seconds=fifo_seconds))
    print(json.dumps({"progress": "serving", **out["runs"][-1]}), file=sys.stderr, flush=True)
    return out


BATCHED_N_INIT = 1000

# The paper's measured runtimes (seconds, one core of an i5-4460, its own C++ code) for
# the 20-bin concentration p.d.f. at eps = 4e-3 (Table of Sec. 6.4, release heights).
PAPER_PDF_SECONDS = {
    50.0: {"StMC-SE": 2561.41, "StMC-GL": 321.77, "StMC-BAOAB": 91.21, "MLMC-SE": 218.52, "MLMC-GL": 265.84},
    100.0: {"StMC-SE": 867.32, "StMC-GL": 277.72, "StMC-BAOAB": 79.25, "MLMC-SE": 120.17, "MLMC-GL": 125.92},
    200.0: {"StMC-SE": 316.33, "StMC-GL": 280.04, "StMC-BAOAB": 78.15, "MLMC-SE": 64.78, "MLMC-GL": 103.69},
}
PDF_BINS = (0.0, 50.0, 20)                       # 20 bins of 0.05 H over [0, H]
PDF_EPS = 4e-3 * PDF_BINS[1] / 1000.0            # RMSE 4e-3 of the density (units 1/H) per bin


def pdf_config(z0, integ):
    """The paper's p.d.f. set-up: release at z0 with U_0 = 0.1 m/s, T = 1000 s, M_0 = 80
    (SE, GL) or 40 (BAOAB), smoothed boxes r = 4, delta = 0.1 H."""
    return W.problem(integrator=integ, z0=float(z0), w0=0.1, release="fixed",
                     M0=40 if integ == "BAOAB" else 80, r=4, delta=100.0)


def pdf_report(ld, precisions=("fp64", "fp32")):
    """MLMC for each integrator and release height, then standard Monte Carlo on the
    finest step MLMC needed (the step the bias test asks for); wall time of each call."""
    import torch
    a0, w, k = PDF_BINS
    rows = []
    for prec in precisions:
        for integ in ("SE", "GL", "BAOAB"):           # warm-up: module load, first allocations
            ld.estimate_pdf(1e-2, pdf_config(100.0, integ), a0, w, k, precision=prec, N_init=1000, L_max=3)
        torch.cuda.synchronize()
        for z0 in (50.0, 100.0, 200.0):
            for integ in ("SE", "GL", "BAOAB"):
                cfg = pdf_config(z0, integ)
                t0 = time.perf_counter()
                m = ld.estimate_pdf(PDF_EPS, cfg, a0, w, k, precision=prec, L_min=2, L_max=12, N_init=10000)
                t_m = time.perf_counter() - t0
                t0 = time.perf_counter()
                st = ld.estimate_pdf(PDF_EPS, cfg, a0, w, k, estimator="stmc", fixed_L=m["L"],
                                     precision=prec, N_init=10000)
                t_s = time.perf_counter() - t0
                for name, r, t in ((f"MLMC-{integ}", m, t_m), (f"StMC-{integ}", st, t_s)):
                    paper = PAPER_PDF_SECONDS[z0].get(name)
                    rows.append({"release_m": z0, "method": name, "precision": prec, "seconds": t,
                                 "paper_seconds": paper, "speedup_vs_paper": (paper / t) if paper else None,
                                 "L": r["L"], "N": r["N"], "fine_steps": r["fine_steps"],
                                 "rmse_est": r["rmse_est"], "status": r["status"],
                                 "density": [p / (w / 1000.0) for p in r["estimate"]]})
                print(json.dumps({"progress": "pdf", **{k2: v for k2, v in rows[-2].items() if k2 != "density"}}),
                      file=sys.stderr, flush=True)
    return rows


ADAPT_X = 50.0                                   # reference height X_adapt (0.05 H)
ADAPT_EPS_REL = (1e-2, 5e-3, 2e-3, 1e-3)


SWEEP_EPS_REL = (1e-2, 3e-3, 1e-3)
SWEEP_Z0 = (100.0, 500.0, 900.0)


def sweep_report(ld):
    """The neutral-layer estimates: release at 100, 500 or 900 m with U_0 ~ N(0,
    sigma_U(z0)^2), T = 1000 s, M_0 = 40, levels up to 9, E[Z(T)] to a relative eps of
    1e-2, 3e-3 or 1e-3, each integrator, FP64 and FP32 paths; wall time per
    mlmc_estimate call (time-to-eps) and the FP32 - FP64 difference in units of eps; and
    standard Monte Carlo (one level) on the finest step the MLMC run needed, FP32."""
    import torch
    rows = []
    for integ in ("SE", "GL", "BAOAB"):
        ld.estimate(1e-2, W.neutral(500.0, integ), precision="fp32", eps_is_relative=True, N_init=1000, L_max=3)
        for z0 in SWEEP_Z0:
            cfg = W.neutral(z0, integ)
            for eps in SWEEP_EPS_REL:
                r = {}
                for prec in ("fp64", "fp32"):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    r[prec] = ld.estimate(eps, cfg, precision=prec, eps_is_relative=True, L_max=9)
                    torch.cuda.synchronize()
                    r[prec]["seconds"] = time.perf_counter() - t0
                a, b = r["fp32"], r["fp64"]
                # standard Monte Carlo on the finest step the MLMC run used (one level of
                # M_0 2^L steps, N by the variance rule), FP32 paths
                st_cfg = dict(cfg, M0=int(cfg["M0"]) << b["L"])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = ld.estimate(eps, st_cfg, precision="fp32", eps_is_relative=True, fixed_L=0)
                torch.cuda.synchronize()
                t_st = time.perf_counter() - t0
                rows.append({"integrator": integ, "z0_m": z0, "eps_rel": eps,
                             "fp64_ms": 1e3 * b["seconds"], "fp32_ms": 1e3 * a["seconds"],
                             "L": b["L"], "N": b["N"], "fine_steps": b["fine_steps"],
                             "estimate_m": b["estimate"], "rmse_est_m": b["rmse_est"],
                             "fp32_minus_fp64_over_eps": (a["estimate"] - b["estimate"]) / b["eps_abs"],
                             "stmc_fp32_ms": 1e3 * t_st, "stmc_fine_steps": st["fine_steps"],
                             "stmc_N": st["N"][0], "stmc_estimate_m": st["estimate"],
                             "status": [a["status"], b["status"], st["status"]]})
                print(json.dumps({"progress": "sweep", **{k: v for k, v in rows[-1].items() if k != "N"}}),
                      file=sys.stderr, flush=True)
    return rows


def adaptive_report(ld, precisions=("fp64", "fp32"), n_bias=1 << 22):
    """Sec. 7 set-up: the mean-position problem (release 50 m, U_0 = 0.1 m/s, T = 1000 s,
    M_0 = 40) with symplectic Euler, uniform against adaptive steps (X_adapt = 50 m):
    E[Y_l] and Var[Y_l] on levels 1..6 from n_bias samples each (the bias of level l is
    about E[Y_{l+1}] / (2^alpha - 1)), then time-to-eps of the adaptive MLMC driver."""
    import torch
    uni = W.problem(integrator="SE", M0=40)
    ada = dict(uni, x_adapt=ADAPT_X)
    levels = list(range(1, 7))
    out = {"levels": [], "runs": []}
    for name, cfg in (("uniform", uni), ("adaptive", ada)):
        ld.estimate(1e-2, cfg, precision="fp64", eps_is_relative=True, N_init=1000, L_max=3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sums = ld.level_sums_batch(cfg, [(l, 0, n_bias) for l in levels], "fp64")
        dt = time.perf_counter() - t0
        for l, s in zip(levels, sums):
            m = s["sum_y"] / s["n"]
            out["levels"].append({"steps": name, "level": l, "mean_Y": m,
                                  "var_Y": s["sum_y2"] / s["n"] - m * m, "n": s["n"]})
        out[f"{name}_level_sums_seconds"] = dt
    for l in levels:
        u = next(r for r in out["levels"] if r["steps"] == "uniform" and r["level"] == l)
        a = next(r for r in out["levels"] if r["steps"] == "adaptive" and r["level"] == l)
        u["bias_ratio_uniform_over_adaptive"] = abs(u["mean_Y"]) / max(abs(a["mean_Y"]), 1e-300)
        u["var_ratio_uniform_over_adaptive"] = u["var_Y"] / max(a["var_Y"], 1e-300)
    for prec in precisions:
        for eps in ADAPT_EPS_REL:
            for name, cfg in (("uniform", uni), ("adaptive", ada)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = ld.estimate(eps, cfg, precision=prec, eps_is_relative=True, N_init=10000,
                                L_min=2, L_max=12)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                out["runs"].append({"precision": prec, "eps_rel": eps, "steps": name, "seconds": t,
                                    "device_seconds": r["device_seconds"], "L": r["L"], "N": r["N"],
                                    "nominal_fine_steps": r["fine_steps"], "estimate": r["estimate"],
                                    "rmse_est": r["rmse_est"], "status": r["status"]})
                print(json.dumps({"progress": "adaptive", **{k: v for k, v in out["runs"][-1].items()
                                                             if k != "N"}}), file=sys.stderr, flush=True)
    return out


def batched_report(ld, steps, warmup, autotune=True):
    """64 independent estimators (mixed release height, tolerance, integrator and QoI)
    in one live engine (ld_engine_run, which submits, steps and collects in the library):
    autotuned FP32 (or the default options), the same options in
    FP64 (also the one-call form that creates its engine), and the same queries one at a
    time through mlmc_estimate in FP64 with a preallocated workspace. Each precision's
    roofline counts the algorithmic operations of every query's coupled steps over the
    engine's kernel time (HIP events around each iteration's graph)."""
    import torch
    spec = W.batched_estimators(64)
    queries = [ld.make_query(q["problem"], q["eps"], eps_is_relative=q["eps_is_relative"],
                             N_init=BATCHED_N_INIT) for q in spec]
    if autotune:
        best, t_tune = ld.autotune(queries, reps=3, precision="fp32")   # median of 3 per configuration
    else:
        best, t_tune = ld.engine_opts(precision="fp32"), 0.0
    res = {}
    for prec in ("fp32", "fp64"):
        o = ld.engine_opts(**dict(ld.opts_dict(best), precision=prec))
        # a live engine, as a server keeps it: its allocation is not timed
        with ld.Engine(o) as eng:
            for _ in range(warmup):
                eng.run(queries)
            torch.cuda.synchronize()
            dev0 = eng.stats()["device_seconds"]
            each = []   # eng.run returns with every result, so each batch is timed whole
            t0 = time.perf_counter()
            for _ in range(steps):
                t1 = time.perf_counter()
                out = eng.run(queries)
                each.append(time.perf_counter() - t1)
            dt = (time.perf_counter() - t0) / steps
            dev_s = (eng.stats()["device_seconds"] - dev0) / steps
        # the one-call form, which creates and frees an engine (about 1 GiB) each time
        t0 = time.perf_counter()
        ld.estimate_batch(queries, opts=o)
        dt_once = time.perf_counter() - t0
        fs = sum(r["fine_steps"] for r in out)
        ops = sum(r["fine_steps"] * FP_OPS_PER_COUPLED_STEP[q["problem"]["integrator"]]
                  for r, q in zip(out, spec))
        achieved = ops / dev_s / 1e12
        res[prec] = {"seconds": dt, "coupled_steps_per_s": fs / dt, "fine_steps": fs,
                     "median_seconds": statistics.median(each), "max_seconds": max(each),
                     "kernel_seconds": dev_s,
                     "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS[prec],
                                  "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[prec],
                                  "peak_unpacked": PEAK_TFLOPS_UNPACKED[prec],
                                  "frac_unpacked": achieved / PEAK_TFLOPS_UNPACKED[prec],
                                  "kernel": ("persistent_kernel" if o.use_graph else "tile_kernel")
                                            + f"<{'float' if prec == 'fp32' else 'double'}, neutral>",
                                  "fp_ops": ops, "coupled_steps": fs, "traffic": None},
                     "one_call_seconds": dt_once,
                     "max_N_l": max(max(r["N"]) for r in out),
                     "min_N_l": min(min(r["N"]) for r in out)}
        if prec == "fp32":
            est32 = [r["estimate"] for r in out]
        else:
            est64 = [r["estimate"] for r in out]
    ws = torch.empty(ld.estimate_workspace_bytes(), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [ld.estimate(q["eps"], q["problem"], precision="fp64", eps_is_relative=q["eps_is_relative"],
                       N_init=BATCHED_N_INIT, workspace=ws, stream=stream) for q in spec]
    t_seq = time.perf_counter() - t0
    res["fp64_one_at_a_time"] = {"seconds": t_seq,
                                 "coupled_steps_per_s": sum(r["fine_steps"] for r in seq) / t_seq}
    # |FP32 - FP64| in units of each query's absolute tolerance
    rel = [abs(a - b) / (q["eps"] * (abs(b) if q["eps_is_relative"] else 1.0))
           for a, b, q in zip(est32, est64, spec)]
    res["fp32_vs_fp64_over_eps_max"] = max(rel)
    res["autotuned"] = {k: v for k, v in ld.opts_dict(best).items() if k != "precision"}
    res["autotune_s"] = t_tune
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="single_large", choices=["single_large", "batched", "serving", "pdf", "adaptive", "sweep"])
    ap.add_argument("--rate", type=float, default=100.0, help="serving: arrivals per second")
    ap.add_argument("--duration", type=float, default=60.0, help="serving: seconds of arrivals")
    ap.add_argument("--fifo-seconds", type=float, default=None,
                    help="serving: stop feeding the FIFO baseline after this many seconds")
    ap.add_argument("--n-init", type=int, default=1000, help="serving: first batch per level")
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="single_large: seconds of the short serving run (0 = none)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--integrator", default="BAOAB", choices=["BAOAB", "GL"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--use-graph", type=int, default=None, choices=[0, 1],
                    help="serving: capture engine iterations in a HIP graph (default: the engine's default)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched: the engine's default options instead of the autotuner's choice")
    ap.add_argument("--plain-schedule", action="store_true",
                    help="single_large: no early top-up (one launch per driver iteration)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB buffer once (scale reference for HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the estimator's samples would shard by "
              "sample range across GPUs, but this build measures the single-GPU path "
              "(--gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1612_07717_amd as ld

    torch.cuda.set_device(0)
    if args.workload == "serving":
        ekw = {} if args.use_graph is None else {"use_graph": bool(args.use_graph)}
        rep = serving_report(ld, args.rate, args.duration, seed=11, n_init=args.n_init,
                             fifo_seconds=args.fifo_seconds, **ekw)
        batch32 = rep["runs"][0]
        print(json.dumps({"metric": "query p50/p99 latency", "value": batch32["p99_ms"],
                          "unit": "ms (p99, FP32 continuous batching)", "n_gpus": 1,
                          "higher_is_better": False, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": f"serving: Poisson arrivals at {args.rate:g} "
                                                 f"queries/s for {args.duration:g} s, release "
                                                 "U[50,950] m, relative eps log-uniform "
                                                 "[3e-4,1e-2], integrator and QoI mixed"},
                          "serving": rep}), flush=True)
        return
    if args.workload == "pdf":
        rows = pdf_report(ld)
        fp64 = [r for r in rows if r["precision"] == "fp64" and r["paper_seconds"]]
        gpu_s = sum(r["seconds"] for r in fp64)
        paper_s = sum(r["paper_seconds"] for r in fp64)
        print(json.dumps({"metric": "time-to-eps of the 20-bin concentration p.d.f. (15 paper runs)",
                          "value": gpu_s, "unit": "s (sum, FP64 paths)", "n_gpus": 1,
                          "higher_is_better": False, "dtype": "f64", "data": "synthetic",
                          "vs_baseline": gpu_s / paper_s,
                          "config": {"workload": "binned concentration, 20 bins of 50 m, r = 4, "
                                                 "delta = 100 m, density RMSE 4e-3, release 50/100/200 m, "
                                                 "U_0 = 0.1 m/s, T = 1000 s, M_0 = 80 (SE, GL) / 40 (BAOAB)",
                                     "paper_seconds_sum": paper_s,
                                     "paper_hardware": "one core of an Intel i5-4460, the paper's C++ code"},
                          "runs": rows}), flush=True)
        return
    if args.workload == "sweep":
        rows = sweep_report(ld)
        total64 = sum(r["fp64_ms"] for r in rows)
        total32 = sum(r["fp32_ms"] for r in rows)
        print(json.dumps({"metric": "time-to-eps, neutral-layer estimates (27 per precision)",
                          "value": total32 / 1e3, "unit": "s (sum, FP32 paths)", "n_gpus": 1,
                          "higher_is_better": False, "dtype": "f32", "data": "synthetic",
                          "vs_baseline": None, "fp64_seconds": total64 / 1e3,
                          "config": {"workload": "neutral layer, z0 100/500/900 m with Gaussian w0, "
                                                 "T = 1000 s, M_0 = 40, L <= 9, relative eps "
                                                 "1e-2/3e-3/1e-3, SE/GL/BAOAB, E[Z(T)]"},
                          "runs": rows}), flush=True)
        return
    if args.workload == "adaptive":
        rep = adaptive_report(ld)
        fp64 = [r for r in rep["runs"] if r["precision"] == "fp64"]
        t_u = sum(r["seconds"] for r in fp64 if r["steps"] == "uniform")
        t_a = sum(r["seconds"] for r in fp64 if r["steps"] == "adaptive")
        print(json.dumps({"metric": "time-to-eps, adaptive over uniform symplectic Euler",
                          "value": t_a / t_u, "unit": "ratio (sum over eps, FP64 paths)", "n_gpus": 1,
                          "higher_is_better": False, "dtype": "f64", "data": "synthetic",
                          "vs_baseline": None,
                          "config": {"workload": "mean position E[X_T]: release 50 m, U_0 = 0.1 m/s, "
                                                 "T = 1000 s, M_0 = 40, X_adapt = 50 m, relative eps "
                                                 + ", ".join(f"{e:g}" for e in ADAPT_EPS_REL)},
                          "adaptive": rep}), flush=True)
        return
    if args.workload == "batched":
        rep = batched_report(ld, args.steps, args.warmup, autotune=not args.no_autotune)
        print(json.dumps({"metric": "coupled particle-steps/s", "value": rep["fp32"]["coupled_steps_per_s"],
                          "unit": "coupled particle-steps/s", "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "ms_per_step": 1e3 * rep["fp32"]["seconds"],
                          "higher_is_better": True, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": "64 estimators: release U[50,950] m, relative eps "
                                                 "log-uniform [1e-3,1e-2], integrator and QoI mixed, "
                                                 "one engine, tiles autotuned"},
                          "roofline": rep["fp32"]["roofline"], "batched": rep}), flush=True)
        return
    cfg = W.single_large(args.integrator)
    L = W.SINGLE_LARGE_LEVELS
    eps = W.SINGLE_LARGE_EPS_REL
    ws = torch.empty(ld.estimate_workspace_bytes(), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    kw = dict(fixed_L=L, eps_is_relative=True, N_init=10000, early_topup=not args.plain_schedule,
              workspace=ws, stream=stream)

    def timed(precision):
        """W untimed then K timed estimates in one precision: (results, seconds)."""
        for _ in range(args.warmup):
            ld.estimate(eps, cfg, precision=precision, **kw)
        torch.cuda.synchronize()
        out = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out.append(ld.estimate(eps, cfg, precision=precision, **kw))
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    def summary(precision, results, elapsed):
        fs = sum(r["fine_steps"] for r in results)
        dev_s = sum(r["device_seconds"] for r in results)
        launches = sum(r["launches"] for r in results)
        return fs, dev_s, launches, roofline(precision, args.integrator, fs, dev_s, launches)

    results, elapsed = timed(args.precision)
    fine_steps, dev_s, launches, roof = summary(args.precision, results, elapsed)
    value = fine_steps / elapsed
    # every integrator step, fine and coarse: sum_l N_l (M_l + M_{l-1}), M_{-1} = 0
    integ_steps = sum(n * ((cfg["M0"] << l) + ((cfg["M0"] << l) >> 1 if l > 0 else 0))
                      for r in results for l, n in enumerate(r["N"]))

    # The same estimate with the other path precision, timed alike, and the error of the
    # run's paths against the other precision's on identical draws and sample counts.
    last = results[-1]
    other = "fp64" if args.precision == "fp32" else "fp32"
    res_o, el_o = timed(other)
    fs_o, dev_o, la_o, roof_o = summary(other, res_o, el_o)
    same = ld.level_sums_batch(cfg, [(l, 0, n) for l, n in enumerate(last["N"])], other)
    est_other_same_n = sum(s["sum_y"] / s["n"] for s in same)
    line = {
        "metric": "coupled particle-steps/s",
        "value": value,
        "unit": "coupled particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "single large estimate: neutral boundary layer, "
                               f"{args.integrator}, z0 = 500 m, Gaussian w0, T = 1000 s, "
                               "dt_0 = T/8, levels 0..12, relative eps 1e-4, E[Z(T)]",
                   "paths": args.precision, "sums": "fp64 compensated",
                   "schedule": "plain" if args.plain_schedule else "early top-up (short levels beside the long ones)",
                   "levels": L + 1, "N_l": last["N"], "fine_steps_per_step": last["fine_steps"],
                   "estimate_m": last["estimate"], "rmse_est_m": last["rmse_est"],
                   "integrator_steps_per_s": integ_steps / elapsed,
                   "time_to_eps_s": last["wall_seconds"], "kernel_s_per_step": dev_s / args.steps,
                   "launches_per_step": launches / args.steps,
                   f"{args.precision}_minus_{other}_same_draws_m": last["estimate"] - est_other_same_n},
        "roofline": roof,
        other: {"value": fs_o / el_o, "unit": "coupled particle-steps/s", "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": 1e3 * el_o / args.steps,
                "time_to_eps_s": res_o[-1]["wall_seconds"], "estimate_m": res_o[-1]["estimate"],
                "N_l": res_o[-1]["N"], "kernel_s_per_step": dev_o / args.steps, "roofline": roof_o},
    }
    if args.serve_seconds > 0:
        rep = serving_report(ld, 100.0, args.serve_seconds, seed=11, n_init=args.n_init)
        line["serving"] = {k: rep[k] for k in ("rate_qps", "duration_s", "arrivals", "N_init")}
        for r in rep["runs"]:
            key = f"{r['policy']}_{r['precision']}"
            line["serving"][key] = {k: r[k] for k in ("p50_ms", "p99_ms", "queries_per_s",
                                                      "coupled_steps_per_s", "max_running")}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(dict(cfg), eps, L, 10000)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
