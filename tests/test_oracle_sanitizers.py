"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host code
only) and driven over small seeded collections by oracle/sanitizer_check.c: no report,
and the checks on the way (output within the candidates and within K by the full edit
distance) hold."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_sanitizer_check")
        subprocess.check_call(["gcc", "-g", "-O1", "-std=gnu11", "-fopenmp",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                               "-fno-omit-frame-pointer", "-Wall", "-o", exe,
                               os.path.join(ROOT, "oracle", "sanitizer_check.c")])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "ok" in r.stdout and "ERROR" not in r.stderr and "runtime error" not in r.stderr
