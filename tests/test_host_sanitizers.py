"""The host runtime's argument checks under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

tests/host_sanitize/driver.cpp calls every C ABI entry point with bad
arguments (and with no device), linked against the host runtime sources
compiled host-only with the sanitizers on the host side (-Xarch_host) and
stub kernel launchers that abort if reached.  Any memory error or undefined
behaviour ends the run with a nonzero status.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2003_02256_amd", "csrc")


def test_host_checks_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "driver")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
    cmd = [hipcc, "--cuda-host-only", "-O1", "-g", "-std=c++17", *san,
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "masw_runtime.hip"), os.path.join(CSRC, "masw_server.hip"),
           "-x", "hip", os.path.join(HERE, "host_sanitize", "driver.cpp"),
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "0 failures" in r.stdout
