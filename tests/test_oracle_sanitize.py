"""The CPU oracle under the address and undefined-behaviour sanitizers
(host code only): a C driver exercises every oracle routine on seeded
random inputs; any out-of-bounds access, leak or undefined operation fails
the run, as does a disagreement between the oracle's merge forms."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_sanitize")
        cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               os.path.join(ROOT, "oracle", "oracle.c"),
               os.path.join(ROOT, "tests", "c", "oracle_sanitize.c"), "-o", exe, "-lm"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "failures 0" in r.stdout
