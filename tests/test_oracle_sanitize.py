"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU): every exported
function on small inputs, empty and clipped cases and every source profile included
(tests/sanitize/oracle_driver.c), must run to its end without a sanitizer report."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc"] + FLAGS + [os.path.join(ROOT, "oracle", "radiate_oracle.c"),
                             os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm", "-o", exe]
    built = subprocess.run(cmd, capture_output=True, text=True)
    if built.returncode != 0 and "sanitize" in built.stderr:
        pytest.skip("gcc here has no sanitizer runtime: " + built.stderr[-200:])
    assert built.returncode == 0, built.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    report = res.stderr
    assert res.returncode == 0, report[-2000:]
    assert "runtime error" not in report and "AddressSanitizer" not in report, report[-2000:]
    assert "checksum" in res.stdout
