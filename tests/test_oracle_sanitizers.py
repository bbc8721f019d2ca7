"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
only): tests/sanitize/oracle_checks.c drives the forward and the VJP over
every profile, directivity and sampling mode and their edge cases; any
out-of-bounds access, leak, overflow or other undefined behaviour fails the
run.  Built with gcc (no OpenMP, so that the sanitizers see plain threads)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_checks")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-Wno-unknown-pragmas", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "sanitize", "oracle_checks.c"),
           os.path.join(ROOT, "oracle", "sbp_oracle.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout and "runtime error" not in r.stderr and "ERROR:" not in r.stderr
