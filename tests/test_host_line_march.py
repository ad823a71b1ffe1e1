"""Host checks of the wetting fill's device helpers (march_line_masked, sincos_quadrant), built
for the CPU from the library's own header by tests/native/line_march_check.cpp."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_masked_march_and_quadrant_sincos(tmp_path):
    cxx = shutil.which("hipcc")
    if cxx is None:
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "line_march_check")
    src = os.path.join(ROOT, "tests", "native", "line_march_check.cpp")
    subprocess.run([cxx, "-O2", "-std=c++17", "-ffp-contract=on",
                    "-I" + os.path.join(ROOT, "paper_2102_04709_amd", "csrc"), "-I" + os.path.join(ROOT, "include"),
                    "-o", exe, src], check=True, capture_output=True)
    r = subprocess.run([exe, "300000"], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
