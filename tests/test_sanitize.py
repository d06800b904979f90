"""Sanitizer builds (CPU only): the oracle, and the host side of the library.

Two small drivers under tests/native/ call every entry point that runs on
the host with arrays of exactly the documented lengths:

* the oracle (oracle/mtvd_oracle.c), built with gcc, AddressSanitizer and
  UndefinedBehaviorSanitizer (OpenMP on, 1-3 threads), on the smallest
  grids its checks accept and on ragged ones, with every switch of the
  scheme;
* the library's host code (the C-ABI functions that do no device work:
  sizes, parameter validation, analysis from row means, boundary layers,
  error strings), built with hipcc for gfx950 with both sanitizers on the
  host side only -- the device code is compiled as usual and never runs
  here.

A report from either sanitizer aborts the driver (no recovery), so the test
checks the exit status and the driver's last line.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
ORACLE = os.path.join(ROOT, "oracle")
CSRC = os.path.join(ROOT, "paper_2411_10372_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

ENV = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:halt_on_error=1:detect_leaks=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, cwd, timeout=300):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=timeout, env=ENV)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    gcc_san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    _run(["gcc", "-std=c99", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer",
          "-ffp-contract=off", "-Wall", "-Wno-unused-function", *gcc_san, "-I", ORACLE,
          "-o", exe, os.path.join(NATIVE, "oracle_sanitize_driver.c"),
          os.path.join(ORACLE, "mtvd_oracle.c"), "-lm"], cwd=str(tmp_path))
    r = _run([exe], cwd=str(tmp_path), timeout=120)
    assert r.stdout.strip().splitlines()[-1] == "oracle sanitize driver ok", r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_host_library_code_under_address_and_undefined_sanitizers(tmp_path):
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    common = ["-O1", "-std=c++17", "-fno-omit-frame-pointer", "--offload-arch=gfx950",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Xarch_host", "-g", *host_san, "-Xarch_host", "-fno-sanitize-recover=all"]
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    srcs.append(os.path.join(NATIVE, "host_sanitize_driver.cpp"))
    objs = [str(tmp_path / (os.path.basename(s) + ".o")) for s in srcs]

    def compile_one(i):
        _run([HIPCC, *common, "-I", os.path.join(ROOT, "include"), "-c", srcs[i],
              "-o", objs[i]], cwd=str(tmp_path))

    with ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(compile_one, range(len(srcs))))
    exe = str(tmp_path / "host_driver")
    _run([HIPCC, "--offload-arch=gfx950", *host_san, *objs, "-o", exe], cwd=str(tmp_path))
    r = _run([exe], cwd=str(tmp_path), timeout=120)
    assert r.stdout.strip().splitlines()[-1] == "host sanitize driver ok", r.stdout
