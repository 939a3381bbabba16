"""The FP64 oracle's C code built with AddressSanitizer and UndefinedBehaviorSanitizer (host
code only) and driven through every entry point on a 4^4 and a ragged 6x4x4x8 lattice
(`tests/sanitize/oracle_driver.c`): no sanitizer report, and the driver's own checks (A
Hermitian, the solvers' success codes and residuals) pass."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "sanitize", "oracle_driver.c"), "-o", exe, "-lm"]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    if build.returncode != 0 and "sanitizer" in build.stderr.lower() and "cannot find" in build.stderr:
        pytest.skip("sanitizer runtime libraries are not installed")
    assert build.returncode == 0, build.stderr[-3000:]
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert "oracle checks passed" in run.stdout
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr
