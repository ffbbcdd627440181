"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
the FP64 oracle (tests/oracle_asan.c drives its 2D and 3D stepping,
trajectories and adjoint with CPML on every face) and the library's launch
plans (tests/plan_check.cpp with plan2d.cpp and plan3d.cpp), built with gcc /
g++ (host code only, no GPU code involved) and run; any sanitizer report
fails the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2405_00814_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-g"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, exe, args=()):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe] + list(args), capture_output=True, text=True, timeout=600, env=ENV)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "orc_asan")
    out = _run(["gcc", "-O1", "-std=c99", "-fopenmp"] + SAN +
               [os.path.join(HERE, "oracle_asan.c"), os.path.join(ROOT, "oracle", "fdtd_oracle.c"),
                "-o", exe, "-lm"], exe)
    assert "oracle sanitizer run: ok" in out


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="g++ or the HIP headers not installed")
def test_plans_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_asan")
    out = _run(["g++", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I", CSRC,
                "-I", os.path.join(ROOT, "include")] + SAN +
               [os.path.join(HERE, "plan_check.cpp"), os.path.join(CSRC, "plan3d.cpp"),
                os.path.join(CSRC, "plan2d.cpp"), "-o", exe], exe, ["5"])
    assert "0 / 1800 bad" in out
