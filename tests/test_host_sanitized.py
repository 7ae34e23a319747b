"""The pure host pieces of the runtime (parameter checks, cutoff table, arena
layout, observables, fault decoding, the autotuner cache) and the request server's scheduling
policy, compiled with g++ under AddressSanitizer and UndefinedBehaviorSanitizer
and run with a fake executor (tests/host/test_host_runtime.cpp).  No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1202_0635_amd", "csrc")


def test_host_runtime_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    exe = str(tmp_path / "host_tests")
    # the sanitizer runtimes are linked statically, so the program runs with
    # whatever the environment preloads
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-static-libasan", "-static-libubsan",
           "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "host", "test_host_runtime.cpp"), os.path.join(CSRC, "sw_host.cpp"),
           "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    cache = tmp_path / "tune_cache.txt"
    cache.write_text("batch gfx950 sites2^10 Lmax2^5 models1 33\nno-value-here\n\nkey-without-number x\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               SWMC_TUNE_CACHE=str(cache))
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "host runtime tests passed" in res.stdout
