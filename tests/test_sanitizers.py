"""CPU-only builds with AddressSanitizer and UndefinedBehaviorSanitizer: the
oracle (g++) and the library's host code (hipcc, sanitizers on the host
side only) each driven by a small program over random and invalid inputs.
A report from either sanitizer fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    os.path.join(HERE, "oracle_driver.cpp"),
                    os.path.join(ROOT, "oracle", "tc_oracle.cpp"), "-o", exe], check=True)
    out = _run(exe)
    assert "oracle driver:" in out


@pytest.mark.skipif(not shutil.which("hipcc") and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_library_host_code_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    csrc = os.path.join(ROOT, "paper_2409_08975_amd", "csrc")
    srcs = [os.path.join(csrc, f) for f in sorted(os.listdir(csrc)) if f.endswith(".hip")]
    exe = str(tmp_path / "abi_driver")
    # sanitizers on the host side only: each -fsanitize= right after -Xarch_host
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer",
           os.path.join(HERE, "abi_driver.cpp")] + srcs + ["-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    out = _run(exe)
    assert "0 failures" in out
