"""Host-side C++ of the library under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

The plain C++ units (1D tables, trace layout, argument validation: the
parts of the C ABI that touch no GPU) are built with g++ together with
host_sanitize_driver.cpp, which runs every degree's tables, every small
mesh and Neumann mask through the layout, and each class of invalid
creation argument through the validation.  The run must print its success
line with no sanitizer report.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2007_11891_amd", "csrc")


def test_host_units_are_clean_under_asan_and_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "host_checks")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "host_setup.cpp"), os.path.join(CSRC, "setup1d.cpp"),
           os.path.join(HERE, "host_sanitize_driver.cpp"), "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    report = run.stdout + run.stderr
    assert run.returncode == 0, report
    assert "host checks OK" in run.stdout, report
    assert "ERROR: AddressSanitizer" not in report and "runtime error" not in report, report
