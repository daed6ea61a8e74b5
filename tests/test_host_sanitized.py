"""The host plan code (plan.cpp, linalg.cpp: octree, lists, FP64 operators,
stage-2 factors, M2L schedule) built with AddressSanitizer and
UndefinedBehaviorSanitizer and run on seeded point sets (no GPU); any invalid
access, leak or undefined operation fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1211_2517_amd", "csrc")


@pytest.mark.parametrize("driver", ["host_plan_check.cpp", "host_ranges_check.cpp"])
def test_host_code_under_sanitizers(tmp_path, driver):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "check")
    flags = ["-O1", "-g", "-std=c++17", "-pthread", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    subprocess.run([gxx, *flags, os.path.join(HERE, driver), os.path.join(CSRC, "plan.cpp"),
                    os.path.join(CSRC, "linalg.cpp"), "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
