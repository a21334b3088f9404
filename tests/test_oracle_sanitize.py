"""The FP64 oracle's C++ under the address and undefined-behaviour sanitizers
(host code only): oracle/sanitize_check.cpp includes the oracle's source and
calls every entry point once on small inputs (render, PSF, error map, log L,
gradient, magnitudes, image-plane source, general multi-plane model). Any
out-of-bounds access, leak or undefined operation aborts the run."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sanitize_check.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_sanitize_check")
        flags = ["-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
                 "-fsanitize=address,undefined"]
        subprocess.run(["g++"] + flags + ["-I", os.path.join(ROOT, "oracle"), SRC, "-o", exe], check=True,
                       capture_output=True, text=True, timeout=300)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "sanitize_check ok" in r.stdout
