"""AddressSanitizer / UndefinedBehaviorSanitizer run of the C oracle (CPU only).

oracle/sanitize_main.c drives every entry point of oracle/schur_pcg.c on small packed
batches; the two files are compiled with gcc under -fsanitize=address,undefined (with
-fno-sanitize-recover, so any report aborts) and leak detection on.  The run must exit 0
and print no sanitizer report.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-std=c99", "-g", "-O1", "-fno-omit-frame-pointer", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ORACLE, "schur_pcg.c"), os.path.join(ORACLE, "sanitize_main.c"),
           "-o", exe, "-lm"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "libasan" in build.stderr:
        pytest.skip("the sanitizer runtime is not installed")
    assert build.returncode == 0, build.stderr
    # verify_asan_link_order=0: the environment may preload a library of its own ahead of
    # the sanitizer runtime; the run leaves the preload list as it is
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    report = run.stdout + run.stderr
    assert run.returncode == 0, report[-4000:]
    assert "runtime error" not in report and "ERROR: AddressSanitizer" not in report, report[-4000:]
    assert "sanitized oracle run ok" in run.stdout
