"""CPU check of the server's host bookkeeping (admission by slot limits and
device memory, the shared device-memory arena, the merge of requests into a
batch, the hand-off of results into each request's buffers) under
AddressSanitizer and UndefinedBehaviorSanitizer, with six threads sharing
one queue and one arena as the server's slot workers do.  The code checked
is the library's own source file, built here with g++ (it makes no HIP
calls)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1302_5507_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_serve_host_under_sanitizers(tmp_path):
    exe = str(tmp_path / "serve_host_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           f"-I{CSRC}", os.path.join(ROOT, "tests", "serve_host_check.cpp"),
           os.path.join(CSRC, "serve_host.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "serve_host_check ok" in r.stdout
