"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/models/oracle_sanitize.c drives every entry point of oracle/bh_ref.h on
inputs that reach all of its branches (every end class, disk, checker and
image sky, fixed-step mode, flat space, caps, radial / zero / non-finite /
out-of-range rays, row and row-list renders).  Built with gcc
-fsanitize=address,undefined and no recovery, so any out-of-bounds access,
leak, use after free, signed overflow, invalid shift or misaligned access
aborts the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = tmp_path / "oracle_san"
    build = subprocess.run(
        ["gcc", "-g", "-O1", "-std=c99", "-fopenmp", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"),
         os.path.join(ROOT, "oracle", "bh_ref.c"), os.path.join(HERE, "models", "oracle_sanitize.c"),
         "-o", str(exe), "-lm"], capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr:
        pytest.skip("this gcc has no sanitizer runtime: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    # (verify_asan_link_order=0: a library preloaded by the environment may
    # come before the sanitizer runtime in the link order)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stderr[-2000:]
    assert "runtime error" not in run.stderr and "ERROR: AddressSanitizer" not in run.stderr
    assert run.stdout.strip().endswith("done")
    # the driver reached every end class
    out = run.stdout
    assert "captured" in out and " disk " in out
