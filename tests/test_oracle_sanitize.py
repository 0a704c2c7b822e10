"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer, driven over
block-boundary sizes, every format, every operator, the statistics and the network
(tests/oracle_host/sanitize_driver.c): no sanitizer report and every round trip exact."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("no host C compiler")
    exe = str(tmp_path / "oracle_sanitize")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", os.path.join(ROOT, "oracle", "ms_oracle.c"),
                    os.path.join(ROOT, "tests", "oracle_host", "sanitize_driver.c"), "-lm", "-o", exe],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "oracle sanitize ok" in r.stdout, r.stderr[-4000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
