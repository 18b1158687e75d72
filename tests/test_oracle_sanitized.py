"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host
code only): a C driver calls every oracle entry point on a small random mask
for both stencils, every collision kind, three cell orders and two
periodicities, and checks sparse AA against dense pull after six steps."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_checked")
    src = os.path.join(HERE, "native", "oracle_checked.c")
    build = subprocess.run(
        ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", src, "-o", exe, "-lm"],
        capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-4000:]
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, (run.stdout + run.stderr)[-4000:]
    assert "max |sparse AA - dense pull|" in run.stdout
