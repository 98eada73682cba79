"""The host code of libaqr (quantiser, graph builder, graph exchange, index
file) built with AddressSanitizer and UndefinedBehaviorSanitizer (g++, no
GPU code) and driven by tests/sanitize/host_driver.cpp on small seeded
inputs and error paths: no sanitizer report, every check passes."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_21600_amd", "csrc")
HOST_SRC = ["errors.cpp", "quantize.cpp", "build.cpp", "indexio.cpp"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_code_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "host_driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-march=x86-64-v3", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-pthread",
           os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
           *[os.path.join(CSRC, s) for s in HOST_SRC], "-o", str(exe)]
    subprocess.run(cmd, check=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe), str(tmp_path)], capture_output=True, text=True, timeout=600,
                       env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr
    assert "0 failures" in r.stdout
