"""Host logic of the stage-2 launch split (no GPU): tile ranges whose chunk
slots stay within the kernel's 32-bit buffer offsets, checked by a small C++
driver against brute force on random schedules."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1211_2517_amd", "csrc")


def test_split_tile_ranges(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "host_ranges_check")
    subprocess.run([gxx, "-O1", "-std=c++17", "-pthread", os.path.join(HERE, "host_ranges_check.cpp"),
                    os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "linalg.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
