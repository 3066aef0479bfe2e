"""The oracle built with AddressSanitizer, UndefinedBehaviorSanitizer and
leak detection, driven through every entry point on a small input with
planted copies, soft-masked runs and N runs (tests/sanitize_oracle.c):
no memory error, undefined behaviour or leak is reported."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_oracle")
    src = [os.path.join(ROOT, "tests", "sanitize_oracle.c"),
           os.path.join(ROOT, "oracle", "sdf_oracle.c"),
           os.path.join(ROOT, "oracle", "sd_align.c")]
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-fopenmp",
                           "-std=c11"] + src + ["-lm", "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out, out
    assert "failures 0" in r.stdout
