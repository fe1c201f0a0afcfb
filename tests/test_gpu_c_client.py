"""The C ABI from C alone: tests/c_client/estimate.c is compiled against
include/ldmlmc.h, linked with libldmlmc.so and run as its own process (no Python in it).
Its estimate and sample counts equal the Python binding's for the same problem."""
import os
import subprocess

import pytest

import paper_1612_07717_amd as ld
import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_c_client_equals_binding(tmp_path):
    exe = tmp_path / "estimate"
    libdir = os.path.join(ROOT, "paper_1612_07717_amd")
    subprocess.run(["gcc", "-O2", "-o", str(exe), os.path.join(ROOT, "tests", "c_client", "estimate.c"),
                    "-I", os.path.join(ROOT, "include"), "-L", libdir, "-lldmlmc",
                    f"-Wl,-rpath,{libdir}"], check=True)
    out = subprocess.run([str(exe), "3e-3"], check=True, capture_output=True, text=True, timeout=120).stdout
    lines = out.split("\n")
    head = lines[0].split()
    c_est = float(head[head.index("estimate") + 1])
    c_N = [int(v) for v in lines[1].split()[1:]]
    cfg = W.neutral(500.0, "BAOAB", M0=40)
    p = ld.estimate(3e-3, cfg, precision="fp64", eps_is_relative=True, N_init=2000, L_max=10)
    assert c_N == p["N"]
    assert c_est == p["estimate"]
