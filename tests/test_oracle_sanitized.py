"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only), driven through every entry point on random small graphs
and update sequences: no out-of-bounds access, leak or undefined behaviour."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "oracle_sanitized"
    srcs = [os.path.join(ROOT, "tests", "oracle_sanitize_driver.cpp"),
            os.path.join(ROOT, "oracle", "kbisim_oracle.cpp"),
            os.path.join(ROOT, "oracle", "maintain_oracle.cpp")]
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-o", str(exe)] + srcs)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.startswith("ok")
