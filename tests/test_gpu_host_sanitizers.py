"""The library's host code under AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer with real device work.

A C client (tests/c_client/host_exercise.c, the C ABI alone) drives the MLMC driver in
both precisions and schedules, the engine (its own API and mlmc_estimate_batch), the
server in both policies and the p.d.f. estimator, linked against the build of the
library whose host code carries the sanitizers (libldmlmc_hostsan.so; its device code
is the product's). Any AddressSanitizer or UndefinedBehaviorSanitizer report fails the
test. Of the leaks LeakSanitizer lists at exit, those allocated from the library's own
code fail it; the HIP runtime's (its code keeps no frame pointers, so their stacks end in
the allocator) are reported only.
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1612_07717_amd")
LIB = os.path.join(PKG, "libldmlmc_hostsan.so")
CLANG = "/opt/rocm/llvm/bin/clang"
REPORT_MARKS = ("runtime error:", "ERROR: AddressSanitizer", "UndefinedBehaviorSanitizer")


def own_leaks(text):
    """LeakSanitizer records whose allocation stack passes through the library."""
    blocks = text.split("leak of ")[1:]
    return [b.split("\n\n")[0] for b in blocks if "libldmlmc_hostsan" in b or "/csrc/" in b]


def test_host_code_under_sanitizers_with_device_work(tmp_path):
    assert os.path.exists(LIB), "libldmlmc_hostsan.so is missing: run __graft_entry__.build()"
    exe = str(tmp_path / "host_exercise")
    subprocess.run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-o", exe,
                    os.path.join(ROOT, "tests", "c_client", "host_exercise.c"), LIB,
                    "-Wl,-rpath," + PKG], check=True)
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libhsakmt\n"
                    "leak:librocprofiler-register\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1",
               LSAN_OPTIONS=f"suppressions={supp}:exitcode=0", UBSAN_OPTIONS="print_stacktrace=1")
    print("case: host_exercise under ASan/LSan/UBSan", flush=True)
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=240)
    sys.stdout.write(r.stdout[-3000:])
    sys.stdout.write(r.stderr[-6000:])
    reports = [ln for ln in (r.stdout + r.stderr).splitlines() if any(m in ln for m in REPORT_MARKS)]
    assert r.returncode == 0 and not reports, (r.returncode, reports[:5])
    assert "host exercise ok" in r.stdout
    leaks = own_leaks(r.stderr)
    assert not leaks, leaks[:3]
