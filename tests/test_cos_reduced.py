"""CPU check of the cosine the oscillatory integrand uses in the kernels
(csrc/cos_reduced.h): the same header compiled for the host and compared
with the C library's cos (tests/cos_reduced_check.cpp): absolute error at
most 4e-16 over [-300, 300], next to multiples of pi/2, near zero and up to
2^20; the library's own result beyond 2^20; NaN for NaN and infinity."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cos_reduced_against_the_c_library(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "cos_check"
    subprocess.run([hipcc, "-O2", "-std=c++17", "-ffp-contract=off",
                    f"-I{os.path.join(ROOT, 'paper_2302_05730_amd', 'csrc')}",
                    os.path.join(ROOT, "tests", "cos_reduced_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
