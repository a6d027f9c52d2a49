"""The host half of the library and the oracle under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only): each is built with its driver in
``tests/sanitize/`` and must run to completion without a report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]


def _build_and_run(cmd, exe, tmp_path):
    if shutil.which(cmd[0]) is None:
        pytest.skip(f"{cmd[0]} not available")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, (out.stdout + out.stderr)[-4000:]
    assert "runtime error" not in out.stderr and "Sanitizer" not in out.stderr, out.stderr[-4000:]
    return out.stdout


def test_host_library_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_driver")
    cmd = ["g++", "-std=c++17"] + SAN + ["-I" + os.path.join(ROOT, "include"),
                                         os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
                                         os.path.join(ROOT, "paper_2608_25376_amd", "csrc", "uavq_host.cpp"),
                                         "-o", exe]
    assert "clean" in _build_and_run(cmd, exe, tmp_path)


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-std=c11"] + SAN + [os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                                       os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe]
    assert "clean" in _build_and_run(cmd, exe, tmp_path)
