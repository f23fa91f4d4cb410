"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, CPU only) and run over its entry points on small seeded problems:
every mode of the E-step, the log-likelihood, the M-step and the EM fit,
including empty input and q = 11."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    src = [os.path.join(ROOT, "tests", "csrc", "oracle_sanitize_main.c"),
           os.path.join(ROOT, "oracle", "cfust_oracle.c")]
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-o", exe] + src + ["-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout[-3000:] + res.stderr[-3000:]
    assert "SANITIZED_OK" in res.stdout
