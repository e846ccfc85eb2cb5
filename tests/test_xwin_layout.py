"""The x-window form's host layout and plan, on the CPU: a check program
built with AddressSanitizer and UBSan regroups random CSR matrices (and the
structural edge cases), verifies every invariant the kernels rely on and
replays both passes on the host against a direct CSR product (no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_xwin_layout_and_plan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "xwin_layout_check"
    build = subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                            "-I", os.path.join(ROOT, "paper_1309_1894_amd", "csrc"),
                            os.path.join(ROOT, "tests", "cpp", "xwin_layout_check.cpp"), "-o", str(exe)],
                           capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr:
        pytest.skip("sanitizer runtime not available")
    assert build.returncode == 0, build.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600,
                         env=dict(os.environ, UBSAN_OPTIONS="halt_on_error=1"))
    assert run.returncode == 0, run.stdout[-4000:] + run.stderr[-4000:]
    assert run.stdout.strip().endswith("ok")
