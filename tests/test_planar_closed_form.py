"""The double pendulum's closed-form dynamics (two point-mass links) in FP64
on the host: equal to the generic planar ABA, reverse equal to central
differences, with joint damping and gravity along both axes.  Compiles the
library's step functions for the host with hipcc."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_closed_form_matches_aba_and_finite_differences(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    exe = tmp_path / "check"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I",
                    os.path.join(ROOT, "paper_2109_08815_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "planar_closed_form_check.hip"), "-o", str(exe)],
                   check=True, capture_output=True, timeout=600)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
