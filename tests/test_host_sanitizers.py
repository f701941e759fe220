"""The library's host-only logic (csrc/host_logic.cpp: argument checks,
serving footprint, batch layouts, row copies) under the address +
undefined-behaviour sanitizers and under the thread sanitizer, on the CPU.

tests/c/host_logic_check.cpp drives it with valid and defective inputs,
random extreme values, and random mixes of serving events packed into
exactly-sized staging and unpacked into exactly-sized result arrays.  The
same source file is compiled into libktf.so; the GPU code is not involved.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "c", "host_logic_check.cpp"),
       os.path.join(ROOT, "paper_1605_05508_amd", "csrc", "host_logic.cpp")]

VARIANTS = {
    "address_undefined": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"],
    "thread": ["-fsanitize=thread"],
}


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_host_logic_sanitized(variant, tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    exe = str(tmp_path / f"host_logic_{variant}")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", *VARIANTS[variant], *SRC, "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stderr}"
    env = dict(os.environ)
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1"
    env["ASAN_OPTIONS"] = "detect_leaks=1:verify_asan_link_order=0"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "host logic OK" in r.stdout, r.stdout + r.stderr
