"""The reverse of a 2D operator as the GPU kernel computes it, checked on the
CPU (no GPU): three cotangent stages fused over tiles of a block's shared
memory against the same reverse written as three whole-grid passes of one
node per thread (`mtvd_adjoint.h`), bit for bit, under AddressSanitizer and
UndefinedBehaviorSanitizer.  The driver (tests/native/adjoint_tile_driver.cpp)
emulates each block's phases in barrier order; see its header for the cases.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2411_10372_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "native", "adjoint_tile_driver.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
@pytest.mark.parametrize("opt", ["-O1", "-O2"])
def test_fused_tiles_equal_the_three_passes(tmp_path, opt):
    exe = str(tmp_path / "adjoint_tile_driver")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"] if opt == "-O1" else []
    r = subprocess.run(["g++", "-std=c++17", opt, "-g", "-ffp-contract=off", "-Wall",
                        "-Wno-unused-function", *san, "-I", CSRC, "-o", exe, DRIVER],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert r.stdout.strip().splitlines()[-1] == "adjoint tile driver ok", r.stdout
