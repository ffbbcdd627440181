"""Host logic: the launch plans (3D single-step and two-steps-per-pass, 2D
multi-step) cover every cell as the kernels require.  Builds
tests/plan_check.cpp with the library's plan sources (host code only) and
runs it on random grids."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2405_00814_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_plan_coverage(tmp_path):
    exe = str(tmp_path / "plan_check")
    cmd = [HIPCC, "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", CSRC, "-I",
           os.path.join(ROOT, "include"), os.path.join(HERE, "plan_check.cpp"),
           os.path.join(CSRC, "plan3d.cpp"), os.path.join(CSRC, "plan2d.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "0 / 9000 bad" in r.stdout
