"""The oracle's C code and the library's host-side table generation built
with AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host code only)
and driven through every entry point on small inputs: any out-of-bounds
access, use after free, leak, overflow of a signed integer or other undefined
behaviour aborts the driver."""
import os
import shutil
import subprocess

import pytest

from oracle import build as obuild

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd_build, exe):
    subprocess.run(cmd_build, check=True, capture_output=True, text=True)
    r = subprocess.run([exe], env=ENV, capture_output=True, text=True, timeout=600)
    if "LeakSanitizer has encountered a fatal error" in r.stderr:
        # the leak checker cannot attach where ptrace is not allowed: run
        # again with the memory-error checks only
        r = subprocess.run([exe], env=dict(ENV, ASAN_OPTIONS="detect_leaks=0"),
                           capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.stdout[-2000:],
                                                                   r.stderr[-4000:])


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    flags = [f for f in obuild.CFLAGS if f not in ("-O2", "-fPIC", "-shared")]
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", *flags, *SAN, "-o", exe, os.path.join(HERE, "sanitize", "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "mco.c"), "-lm"], exe)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_tables_under_sanitizers(tmp_path):
    exe = str(tmp_path / "tables_driver")
    _run(["g++", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", *SAN, "-o", exe,
          os.path.join(HERE, "sanitize", "tables_driver.cpp"),
          os.path.join(ROOT, "paper_2201_13191_amd", "csrc", "tables.cpp")], exe)
