"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

- The oracle is rebuilt with gcc's sanitizers and its fast pin tests run against that
  build (every oracle function they reach: Philox, normals, steps, couplings, adaptive
  samples, sums, planners, the driver).
- The library is rebuilt with clang's sanitizers on its host code only (the device code
  is compiled as usual) and the host-logic tests run against it: the planners, argument
  validation, the engine's and server's checks that precede device use, the bench
  helpers.

Each child run loads the sanitizer runtime first; any report ends it with a non-zero
status and the report in its output. Leak checking is off: the children are Python
processes, whose own allocations at exit would drown the library's.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer"]
REPORT_MARKS = ("runtime error:", "AddressSanitizer", "UndefinedBehaviorSanitizer")


def _run(cmd, env, timeout):
    r = subprocess.run(cmd, env=env, cwd=ROOT, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    reports = [ln for ln in out.splitlines() if any(m in ln for m in REPORT_MARKS)]
    assert r.returncode == 0 and not reports, (r.returncode, reports[:5], out[-3000:])
    return out


@pytest.mark.slow
def test_oracle_pins_under_sanitizers(tmp_path):
    import oracle
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    oracle.build(out=lib, extra_flags=FLAGS)
    env = dict(os.environ, LD_ORACLE_LIB=lib, LD_PRELOAD=libasan, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")
    files = ["test_oracle_rng.py", "test_oracle_philox_independent.py", "test_oracle_model.py",
             "test_oracle_closed_forms.py", "test_oracle_adaptive.py",
             "test_oracle_smoothing_sums_driver.py", "test_oracle_pdf.py"]
    out = _run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider",
                "-m", "not slow and not gpu"] + [os.path.join(ROOT, "tests", f) for f in files],
               env, timeout=900)
    assert " passed" in out


@pytest.mark.slow
def test_library_host_code_under_sanitizers(tmp_path):
    from paper_1612_07717_amd import build as libbuild
    rts = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rts:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    # the in-tree sanitizer build if it is current, else a fresh one
    lib = libbuild.HOSTSAN_LIB if libbuild.hostsan_is_current() else \
        libbuild.build(out=str(tmp_path / "libldmlmc_san.so"), host_flags=libbuild.HOSTSAN_FLAGS)
    env = dict(os.environ, LDMLMC_LIB=lib, LD_PRELOAD=rts[-1],
               ASAN_OPTIONS="detect_leaks=0:alloc_dealloc_mismatch=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    out = _run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider",
                "-m", "not gpu", os.path.join(ROOT, "tests", "test_lib_host.py"),
                os.path.join(ROOT, "tests", "test_bench_host.py")], env, timeout=900)
    assert " passed" in out
