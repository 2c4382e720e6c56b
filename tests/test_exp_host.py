"""The HIP path's FP64 exponential, checked on the host: the header that
defines it is compiled for the CPU with the C library's fma (the same
operations in the same order; the device build only picks the instruction
form of each multiply-add)."""
import os

import pytest


def test_library_exp_f64_within_one_ulp(tmp_path):
    """The HIP path's FP64 exponential (Cody-Waite reduction, degree-13
    polynomial, one scaling), built for the host from the same header,
    stays within one ulp of the long-double exponential over x in
    [-745, 0], subnormal results included."""
    import shutil
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "exp_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-ffp-contract=off",
                    "-I", os.path.join(root, "paper_2506_09743_amd", "csrc"),
                    os.path.join(root, "tests", "helpers", "exp_f64_check.cpp"), "-o", exe], check=True)
    for lo, n in ((-745.0, 3000000), (-1.0, 1000000), (-1e-6, 200000)):
        worst, worst_x, checked = subprocess.run([exe, str(lo), str(n)], capture_output=True, text=True,
                                                 check=True).stdout.split()
        print(f"exp_f64 on [{lo}, 0]: max error {float(worst):.3f} ulp at x = {worst_x} ({checked} arguments)")
        assert float(worst) <= 1.0
