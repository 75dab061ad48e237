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


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_fft_plans_are_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    # the same check built with AddressSanitizer and UBSan: every register
    # array index of the stage code (values, twiddle powers) and every
    # exchange position stays in bounds for every plan (an out-of-range
    # twiddle power, say, stops the run with a runtime error)
    exe = str(tmp_path / "fft_plan_check_san")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I" + os.path.join(HERE, "host"), "-I" + CSRC,
           os.path.join(HERE, "host", "fft_plan_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and ("asan" in r.stderr or "ubsan" in r.stderr):
        pytest.skip("sanitizer runtimes not installed: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
