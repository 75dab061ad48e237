"""The kernels' FFT plans on the CPU: tests/host/fft_plan_check.cpp compiles
the device FFT header (radix codelets, stage twiddles, the per-thread
Stockham positions) with g++ and runs each plan's cooperating threads one
after another against the DFT written out as a sum, forward and inverse,
for every transform length of the library.  A wrong radix codelet, twiddle
power or exchange position gives O(1) errors; correct plans agree to a few
ulp."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_0911_1407_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_fft_plans_match_the_dft_on_the_host(tmp_path):
    exe = str(tmp_path / "fft_plan_check")
    cmd = ["g++", "-O1", "-std=c++17", "-I" + os.path.join(HERE, "host"), "-I" + CSRC,
           os.path.join(HERE, "host", "fft_plan_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = [l for l in r.stdout.splitlines() if l.startswith("N=")]
    # 12 lengths, forward and inverse
    assert len(lines) == 24 and all(l.endswith(" ok") for l in lines), r.stdout
