"""Host-only check of the plan builder's device addresses (no GPU needed).

Builds tests/host/plan_check.cpp against the library's host sources with g++
and runs it: every pack slot names a real term of its own problem, every
reduce item stays inside its problem's row arrays, and every compact-basis
row is finished by exactly one item, across schedules and multi-problem
plans.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2111_13655_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")),
                    reason="needs g++ and the HIP headers")
def test_plan_device_addresses(tmp_path):
    exe = str(tmp_path / "plan_check")
    cmd = ["g++", "-std=c++17", "-O1", "-I" + os.path.join(ROCM, "include"), "-I" + CSRC,
           "-D__HIP_PLATFORM_AMD__", os.path.join(ROOT, "tests", "host", "plan_check.cpp")]
    cmd += [os.path.join(CSRC, f) for f in ("sg_plan.cpp", "sg_terms.cpp", "sg_tables.cpp")]
    cmd += ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
            "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:]
    assert "0 bad" in r.stdout
