"""Builds libldmlmc.so (HIP kernels + host runtime + C ABI) for gfx950 with hipcc.

    python -m paper_1612_07717_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libldmlmc.so")
SOURCES = ["kernels.hip", "api.cpp", "driver.cpp", "engine.cpp", "server.cpp", "pdf.cpp", "smoothing.cpp"]

# -packed-fp32-ops: never emit v_pk_{add,mul,fma}_f32 (packed FP32 has given silent
# wrong results on these boxes). No fast-math: the compensated sums and the expm1-based
# O-step rely on IEEE semantics. -ffp-contract=on: a multiply feeds an add as one FMA only
# within one source expression (a * b + c), never across statements, so every inlined
# copy of a step rounds alike (HIP's default, fast, lets the backend choose per context).
HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-fno-fast-math", "-ffp-contract=on", "-Wall", "-Wno-unused-function"]


# The same library with AddressSanitizer and UndefinedBehaviorSanitizer in its host code
# (every flag goes behind -Xarch_host; the device code is the product's). A GPU test runs
# a C client against it that drives the driver, the engine, the server and the p.d.f.
# estimator.
HOSTSAN_LIB = os.path.join(HERE, "libldmlmc_hostsan.so")
HOSTSAN_FLAGS = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
                 "-fno-omit-frame-pointer", "-g"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False, out: str = LIB, host_flags=()) -> str:
    """Compile every source into one shared library at `out`. Each of `host_flags` is
    passed to the host compilation only (behind -Xarch_host); device code is unchanged."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp"
    host = [a for f in host_flags for a in ("-Xarch_host", f)]
    cmd = [hipcc()] + HIPCC_FLAGS + host + ["-I", os.path.join(ROOT, "include"), "-o", tmp] + srcs
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines()
            if "packed-fp32-ops' is not a recognized feature" not in ln]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(tmp, out)
    return out


def build_hostsan(verbose: bool = False) -> str:
    return build(verbose=verbose, out=HOSTSAN_LIB, host_flags=HOSTSAN_FLAGS)


def hostsan_is_current() -> bool:
    """True if the sanitizer build exists and is newer than every source and header."""
    if not os.path.exists(HOSTSAN_LIB):
        return False
    inputs = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + \
             [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    return os.path.getmtime(HOSTSAN_LIB) >= max(os.path.getmtime(f) for f in inputs)


if __name__ == "__main__":
    print(build(verbose=True))
