"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the host code on the CPU: the FP64
oracle (g++), driven through every boundary type and its rejected inputs, and the library's host
set-up and validation (lbm3_workspace_bytes, built with hipcc with the sanitizers on the host pass
only; no device call is made).  Any sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=ENV)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    assert "ALL OK" in r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path / "oracle_sanitize")
    subprocess.run([gxx, "-std=c++17", "-fopenmp", *SAN, "-o", exe, os.path.join(ROOT, "tests", "native", "oracle_sanitize.cpp"),
                    os.path.join(ROOT, "oracle", "lbm3_oracle.cpp")], check=True, capture_output=True)
    _run(exe)


def test_library_host_setup_under_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "plan_sanitize")
    csrc = os.path.join(ROOT, "paper_2102_04709_amd", "csrc")
    host_san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined"):
        host_san += ["-Xarch_host", f]
    cmd = [hipcc, "--offload-arch=gfx950", "-std=c++17", "-O1", "-g", *host_san,
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-I" + csrc, "-o", exe,
           os.path.join(ROOT, "tests", "native", "plan_sanitize.cpp"),
           os.path.join(csrc, "lbm3_api.cpp"), os.path.join(csrc, "lbm3_kernels.hip"), os.path.join(csrc, "lbm3_adjoint.hip")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    _run(exe)
