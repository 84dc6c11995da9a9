"""Host-only builds of the serving scheduler and of the oracle, run on the CPU.

- The scheduler of ``gut_serve_*`` (``serve_core.h``) is driven by a fake
  device backend (``tests/host/serve_core_test.cpp``): arena, admission,
  batch formation, pair-buffer growth under contention (two slots whose grown
  pair buffers cannot both fit), batch splitting, error paths and statistics.
  It is built plainly, under AddressSanitizer + UndefinedBehaviorSanitizer and
  under ThreadSanitizer.
- Every entry point of the FP64 oracle runs under AddressSanitizer +
  UndefinedBehaviorSanitizer (``tests/host/oracle_sanitize.c``).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
INC = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2412_12507_amd", "csrc")]

SAN = {
    "plain": [],
    "asan_ubsan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"],
    "tsan": ["-fsanitize=thread"],
}


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=env)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
@pytest.mark.parametrize("mode", list(SAN))
def test_serve_scheduler_host(tmp_path, mode):
    exe = str(tmp_path / f"serve_core_{mode}")
    _run(["g++", "-std=c++17", "-O1", "-g", "-pthread"] + SAN[mode] + INC +
         [os.path.join(HOST, "serve_core_test.cpp"), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", TSAN_OPTIONS="halt_on_error=1")
    out = _run([exe], env=env)
    assert "ALL OK" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    _run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp"] + SAN["asan_ubsan"] +
         ["-I", os.path.join(ROOT, "oracle"), os.path.join(HOST, "oracle_sanitize.c"),
          os.path.join(ROOT, "oracle", "oracle.c"), "-o", exe, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="4")
    out = _run([exe], env=env)
    assert "oracle sanitize ok" in out
