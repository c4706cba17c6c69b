"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only): a driver calls every entry point on small lattices -- the
clover term, the operator (whole lattice and sites), D_BB, both block solves,
both SAP forms, FGMRES to 1e-10 -- and checks the invalid-argument paths.
Any out-of-bounds access, leak or undefined behaviour makes the sanitized
binary exit non-zero."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fcx-fortran-rules", "-I" + ORACLE,
           os.path.join(HERE, "oracle_sanitize_driver.c"), os.path.join(ORACLE, "oracle.c"), "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr
