"""The serving loop's host copy pool, on the CPU: a stress program built with
ThreadSanitizer copies random batches through pools with and without worker
threads and checks every byte (no GPU involved)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_copy_pool_under_thread_sanitizer(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "copy_pool_stress"
    build = subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
                            "-I", os.path.join(ROOT, "paper_1309_1894_amd", "csrc"),
                            os.path.join(ROOT, "tests", "cpp", "copy_pool_stress.cpp"), "-o", str(exe)],
                           capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr:
        pytest.skip("ThreadSanitizer runtime not available")
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:exitcode=66")
    run = subprocess.run([str(exe), "60"], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.strip().endswith("ok")
