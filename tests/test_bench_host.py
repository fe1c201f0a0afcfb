"""Host checks of bench.py's bookkeeping (no GPU).

- kernel_hash finds the dominant kernel's machine code in the built library, gives
  different hashes for different kernels and 'missing' for an unknown symbol;
- the committed counter summaries carry a hash of the same form.
"""
import json
import os
import re

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1612_07717_amd", "libldmlmc.so")


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_kernel_hash_reads_the_code_object():
    h32 = bench.kernel_hash()
    h64 = bench.kernel_hash("_ZN3ldm12level_kernelIdLi2ELi1EEEvNS_5KArgsEP13ld_level_sumsPd")
    assert re.fullmatch(r"[0-9a-f]{16}", h32) and re.fullmatch(r"[0-9a-f]{16}", h64)
    assert h32 != h64
    assert bench.kernel_hash("no_such_kernel") == "missing"


def test_committed_summaries_carry_a_kernel_hash():
    for name in ("level_kernel_fp32_single_large_traffic.json", "level_kernel_fp32_single_large_valu.json",
                 "level_kernel_fp64_single_large_traffic.json", "level_kernel_fp64_single_large_valu.json"):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            d = json.load(f)
        assert re.fullmatch(r"[0-9a-f]{16}", d["kernel_hash"])


def test_roofline_follows_the_per_step_operation_count():
    """achieved = operations per coupled fine step (70 FP ALU + 13 elementary functions
    for BAOAB) x coupled steps / kernel seconds; frac against 157.3 TFLOP/s (packed FP32)
    and 78.6 (unpacked FP32, and FP64)."""
    r = bench.roofline("fp32", "BAOAB", 8.34e8, 6.6e-3, 4)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["fp_ops_per_coupled_step"] == 83.0 and r["int_ops_per_coupled_step"] == 25.0
    assert abs(r["achieved"] - 83.0 * 8.34e8 / 6.6e-3 / 1e12) < 1e-12
    assert abs(r["frac"] - r["achieved"] / 157.3) < 1e-15
    assert abs(r["frac_unpacked"] - r["achieved"] / 78.6) < 1e-15
    assert abs(r["avg_launch_ms"] - 1.65) < 1e-12
    r64 = bench.roofline("fp64", "GL", 1e9, 1e-2, 2)
    assert r64["peak"] == 78.6 and abs(r64["achieved"] - 6.0) < 1e-12
