"""The oracle built with the address and undefined-behaviour sanitizers.

oracle/sanitize_driver.c compiles the whole oracle into one program and
runs coupled steps through every entry point the parity tests use: the
linear spring-dashpot with the Lagrange gather (D2Q9), Hertz-Mindlin
contacts (no-slip and micro-slip) with rotation, a tangential history
carried over three steps and fixed obstacle points with their own areas
(D3Q19), Hertz with fixed points
(D2Q9), soft repulsion with bins of four cells (D3Q15), a periodic lattice,
and both candidate searches.  Any out-of-bounds access, use after free,
leak, signed overflow, bad shift or float-to-int overflow aborts the
program with a report.  The node loops run on several threads.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(os.path.dirname(HERE), "oracle", "sanitize_driver.c")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    flags = ["-O1", "-g", "-std=c99", "-fopenmp", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    subprocess.check_call(["gcc", *flags, DRIVER, "-o", exe, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="3")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr
    assert r.stdout.strip().endswith("sanitize_driver: ok")
    lines = r.stdout.splitlines()
    assert "history 0, skin" not in lines[1] and "history 0, skin" not in lines[2]   # Hertz-Mindlin carried contacts
