"""The host half of the kernels' division by a launch-wide divisor
(hjx_fastdiv.h): a C++ checker compiled with g++ compares the multiplier's
quotients with integer division over whole ranges, and checks that it is
refused where it would not be exact."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_fast_div_multiplier_is_exact(tmp_path):
    exe = str(tmp_path / "fastdiv_check")
    subprocess.run(["g++", "-std=c++17", "-O2", os.path.join(HERE, "native", "fastdiv_check.cpp"), "-o", exe],
                   check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert ", 0 wrong" in r.stdout
