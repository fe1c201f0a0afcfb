"""Benchmark: coupled particle-steps/s of the MLMC dispersion hot path on one MI355X.

One step = one full adaptive MLMC estimate (all levels, the driver's iterations, the
level kernels and the FP64 planning) of the large single-estimate workload: neutral
boundary layer, BAOAB, release at 500 m with Gaussian w0, T = 1000 s, dt_0 = T/8,
levels 0..12, relative eps 1e-4, E[Z(T)], FP32 paths with FP64 compensated sums.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32|fp64]

Prints one JSON line. The CPU baseline times the oracle on a bounded sample of the
same workload on this host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

# Peak figures of one MI355X (public): 256 CUs at 2.4 GHz. FP32 vector 157.3 TFLOP/s
# (packed FMA: 256 FLOP/clk/CU); FP64 vector 78.6 TFLOP/s (128 FLOP/clk/CU).
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}

# Arithmetic operations the method performs per coupled fine step (one fine step, half
# a coarse step, half a coupling, half a Philox block, one normal), counted from the
# equations: +, -, *, compare, min/max, select and integer ops count 1, a multiply-add
# counts 2, each elementary function (sqrt, reciprocal, expm1, log, sin, cos) counts 1.
# Breakdown in DESIGN.md ("Algorithmic work per coupled step").
OPS_PER_COUPLED_STEP = {
    ("BAOAB", "neutral"): 135.5, ("GL", "neutral"): 119.0, ("SE", "neutral"): 115.5,
    ("BAOAB", "homogeneous"): 91.0, ("GL", "homogeneous"): 84.5, ("SE", "homogeneous"): 83.5,
}

KERNEL_SOURCES = ["paper_1612_07717_amd/csrc/kernels.hip", "paper_1612_07717_amd/csrc/device_model.hpp",
                  "paper_1612_07717_amd/csrc/device_rng.hpp", "paper_1612_07717_amd/csrc/ld_internal.hpp"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def hbm_traffic(precision: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None when
    the summary is missing or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"level_kernel_{precision}_single_large_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except OSError:
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(cfg, N_levels, target_steps=2.5e8):
    """The oracle on a bounded sample: each level's samples scaled down by the same
    factor so the sample has about target_steps coupled fine steps."""
    import oracle
    total = sum(n * (cfg["M0"] << l) for l, n in enumerate(N_levels))
    f = min(1.0, target_steps / total)
    counts = [max(64, int(n * f)) for n in N_levels]
    steps = sum(n * (cfg["M0"] << l) for l, n in enumerate(counts))
    t0 = time.perf_counter()
    for l, n in enumerate(counts):
        oracle.level_sums(cfg, l, 0, n)
    dt = time.perf_counter() - t0
    return {"value": steps / dt, "unit": "coupled particle-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"levels 0..{len(counts) - 1} of the same workload with N_l scaled by "
                      f"{f:.3g} (N_l = {counts}), {steps:.3g} coupled fine steps, FP64, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--integrator", default="BAOAB", choices=["BAOAB", "GL"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    cfg = W.single_large(args.integrator)
    L = W.SINGLE_LARGE_LEVELS
    eps = W.SINGLE_LARGE_EPS_REL
    ws = torch.empty(ld.estimate_workspace_bytes(), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    kw = dict(precision=args.precision, fixed_L=L, eps_is_relative=True, N_init=10000,
              workspace=ws, stream=stream)

    for _ in range(args.warmup):
        ld.estimate(eps, cfg, **kw)
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        results.append(ld.estimate(eps, cfg, **kw))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    fine_steps = sum(r["fine_steps"] for r in results)
    value = fine_steps / elapsed

    # The same estimate with all-FP64 paths (time-to-eps), and the FP32 run's error
    # against FP64 paths on identical draws and sample counts.
    last = results[-1]
    other = "fp64" if args.precision == "fp32" else "fp32"
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r_other = ld.estimate(eps, cfg, **dict(kw, precision=other))
    torch.cuda.synchronize()
    t_other = time.perf_counter() - t1
    same = ld.level_sums_batch(cfg, [(l, 0, n) for l, n in enumerate(last["N"])], other)
    est_other_same_n = sum(s["sum_y"] / s["n"] for s in same)
    dev_s = sum(r["device_seconds"] for r in results)
    launches = sum(r["launches"] for r in results)
    ops = OPS_PER_COUPLED_STEP[(args.integrator, cfg["profile"])]
    achieved = ops * fine_steps / dev_s / 1e12
    peak = PEAK_TFLOPS[args.precision]
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
                   "levels": L + 1, "N_l": last["N"], "fine_steps_per_step": last["fine_steps"],
                   "estimate_m": last["estimate"], "rmse_est_m": last["rmse_est"],
                   "time_to_eps_s": last["wall_seconds"], "kernel_s_per_step": dev_s / args.steps,
                   "launches_per_step": launches / args.steps,
                   f"time_to_eps_{other}_s": t_other,
                   f"estimate_{other}_m": r_other["estimate"],
                   f"{args.precision}_minus_{other}_same_draws_m": last["estimate"] - est_other_same_n},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": hbm_traffic(args.precision),
                     "kernel": f"level_kernel<{'float' if args.precision == 'fp32' else 'double'}>",
                     "ops_per_coupled_step": ops,
                     "avg_launch_ms": 1e3 * dev_s / launches},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(dict(cfg), last["N"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
