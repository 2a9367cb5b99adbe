"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/native/oracle_sanitize.c includes oracle.c and calls every entry point
on small geometries (odd and even sizes, rays on pixel edges, bins missing
the image, subsampled angles, one pixel, one angle), including a NaN in the
data that must stop every inner CG solve at its first step (a breakdown)
and leave the image at zero.  Any out-of-bounds access, use after free, leak
or undefined behaviour aborts the run.  CPU only (gcc)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_sanitize")
    subprocess.run([gcc, "-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fopenmp",
                    "-ffp-contract=off", os.path.join(HERE, "native", "oracle_sanitize.c"), "-o", exe,
                    "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count(" ok") == 8, r.stdout
