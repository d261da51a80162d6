"""The host-side C and C++ code under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU: the pool builder of the library
(rg_build_host.cpp, compiled for the host only) and the CPU oracle with the
input generator. Each is built with the sanitizers into a temporary
directory and run on checks written beside it (tests/native/); any
out-of-bounds access, leak or undefined behaviour fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, env=ENV)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr[-4000:]}"
    return r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_pool_builder_under_sanitizers(tmp_path):
    exe = str(tmp_path / "pool_builder_check")
    # host-only compilation: the sanitizers apply to host code
    _run([HIPCC, "-x", "hip", "--cuda-host-only", "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=address",
          "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
          "-I", os.path.join(ROOT, "paper_1709_07821_amd", "csrc"), os.path.join(NATIVE, "pool_builder_check.cpp"),
          os.path.join(ROOT, "paper_1709_07821_amd", "csrc", "rg_build_host.cpp"), "-o", exe], str(tmp_path))
    out = _run([exe], str(tmp_path))
    assert "all checks passed" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_and_generator_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          os.path.join(NATIVE, "oracle_check.c"), os.path.join(ROOT, "oracle", "oracle.c"),
          os.path.join(ROOT, "synth", "synth.c"), "-lm", "-o", exe], str(tmp_path))
    out = _run([exe], str(tmp_path))
    assert "all checks passed" in out
