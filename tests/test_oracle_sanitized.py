"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host only): tests/oracle_sanitize_driver.c calls every entry point on
random graphs, including the empty graph and a trace capacity that is too
small, and checks the certificate of the oracle's own cores."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_clean_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_sanitize")
    build = subprocess.run([gcc, "-g", "-O1", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
                            "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined",
                            os.path.join(HERE, "oracle_sanitize_driver.c"),
                            os.path.join(ROOT, "oracle", "khc_oracle.c"), "-o", exe],
                           capture_output=True, text=True)
    if build.returncode != 0 and "asan" in build.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert "oracle sanitizer run ok" in run.stdout
