"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code
(CPU only): the FP64 oracle driven through every entry point, and the host
side of the C ABI (validation, layouts, context life cycle, call order) in a
build whose host code carries both sanitizers (device code unchanged, never
launched).  A report from either sanitizer fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fopenmp",
                           "-o", exe, os.path.join(SAN, "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "sobrc_oracle.c"), "-lm"])
    assert "all calls returned" in _run(exe)


HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_abi_host_code_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "abi_san")
    csrc = os.path.join(ROOT, "paper_1403_0240_amd", "csrc")
    # the sanitizers apply to the host pass only (-Xarch_host before each)
    subprocess.check_call([HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-Xarch_host", "-fno-omit-frame-pointer",
                           "-I", os.path.join(ROOT, "include"), "-I", csrc,
                           os.path.join(SAN, "abi_driver.cpp"), os.path.join(csrc, "sobrc_abi.hip"),
                           os.path.join(csrc, "sobrc_kernels.hip"), os.path.join(csrc, "sobrc_deconv.hip"),
                           "-o", exe], stderr=subprocess.DEVNULL)
    assert "all host-side checks passed" in _run(exe)
