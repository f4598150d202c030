"""The planner (csrc/plan.cpp, pure host code) under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/plan_check.cpp plans a matrix of problems (every precision and contraction form, crop windows
and full cells, interp_f 1 .. 4, 384 and power-of-two grids, slice groups at the smallest accepted
budget and with S_1 checkpoints, resident S-matrices, the inverse multislice, companion images, invalid problems) and checks
every table of each plan against the buffers the device path binds it to.  Built with g++ (host
code only, no device code), so it runs without a GPU.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_planner_under_asan_and_ubsan(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path / "plan_check")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1908_07628_amd", "csrc"),
           os.path.join(ROOT, "tests", "plan_check.cpp"),
           os.path.join(ROOT, "paper_1908_07628_amd", "csrc", "plan.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-6000:]
    assert "cases ok" in r.stdout
    # the matrix reached every form it is meant to cover
    for what in ("raster", "window-Gram", "Gram", "with slice groups", "with S_1 checkpoints"):
        m = re.search(r"(\d+) %s[,;]" % re.escape(what), r.stdout)
        assert m and int(m.group(1)) > 0, (what, r.stdout)
