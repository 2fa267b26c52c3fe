"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a
driver (tests/oracle_sanitize_driver.c) calls every oracle entry point on
small seeded inputs with exactly sized buffers, built with gcc
-fsanitize=address,undefined; any out-of-bounds access, leak or undefined
behaviour aborts the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "orc_sanitized")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-o", exe,
                           os.path.join(HERE, "oracle_sanitize_driver.c"), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized oracle: 72 cases" in r.stdout
