"""The host half of the library (ranges, amounts, orders) built on its own
with AddressSanitizer and UndefinedBehaviorSanitizer and driven through the
C ABI on valid and invalid arguments (tests/host/sanitize_driver.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1302_6189_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "host", "sanitize_driver.cpp"),
           os.path.join(CSRC, "decomp.cpp"), os.path.join(CSRC, "capi_host.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, timeout=600)
    # verify_asan_link_order=0: the sanitizer runtime need not come first among
    # libraries the environment preloads
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip().endswith("ok")
