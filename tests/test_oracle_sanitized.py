"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, CPU only) and driven through every entry point by
tests/sanitize_oracle_main.c: no invalid access, no undefined operation,
and every call returns what it should."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
FLAGS = ["-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall", "-Wno-unknown-pragmas"]


@pytest.mark.slow
def test_oracle_runs_clean_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "sanitized_oracle")
    subprocess.run([gcc, *FLAGS, "-o", exe, os.path.join(HERE, "sanitize_oracle_main.c"), "-lm"],
                   check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "sanitized oracle run: ok" in r.stdout
