"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/sanitize_driver.c includes the oracle's source and runs it on small
synthetic scenes (periodic boxes with a free solid in 2D and 3D, both
materials, one shared step, the velocity-based contrast, a floor with a
clamped post); any invalid access, leak or undefined operation aborts it.
Host code only, built with gcc.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_runs_clean_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    exe = str(tmp_path / "sanitize_driver")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wno-unknown-pragmas",
           "-o", exe, os.path.join(HERE, "sanitize_driver.c"), "-lm"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr and "cannot find" in build.stderr:
        pytest.skip("sanitizer runtime not installed")
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 6 and all(l.endswith(" ok") for l in lines), r.stdout
    # the scenes did rebuild and sub-step
    assert all(" rebuilds 0 " not in l for l in lines), r.stdout
