"""Sanitizer builds of the CPU code: the C oracle and the library's host-side
layout and work-list code, compiled with AddressSanitizer and
UndefinedBehaviorSanitizer (host compilers only) and run on small odd shapes."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-O1", "-g"]


def _build_and_run(cmd, exe):
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    out = _build_and_run(["gcc", *SAN, "-std=c11", "-ffp-contract=off",
                          os.path.join(ROOT, "oracle", "lbm_oracle.c"),
                          os.path.join(ROOT, "tests", "sanitize", "oracle_main.c"), "-o", exe, "-lm"], exe)
    assert "0 unexpected results" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_host_layout_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "host_san")
    out = _build_and_run(["g++", *SAN, "-std=c++17", "-I",
                          os.path.join(ROOT, "paper_1204_4098_amd", "csrc"),
                          os.path.join(ROOT, "tests", "sanitize", "host_main.cpp"), "-o", exe], exe)
    assert "0 failed checks" in out
