"""AddressSanitizer + UndefinedBehaviorSanitizer builds (CPU only, gcc/g++) of the oracle's C
part and of the library's host-only source (cosmology factors, halt predicate, forecast),
each driven through every function on small inputs: no sanitizer finding, expected status
codes.  The GPU kernels are outside this check (no device sanitizer on this hardware)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def _run(cmd_build, exe, tmp_path):
    r = subprocess.run(cmd_build, capture_output=True, text=True, cwd=tmp_path)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc needed")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    out = _run(["gcc", *SAN, "-fopenmp", "-ffp-contract=off", "-o", exe,
                os.path.join(ROOT, "oracle", "dzs_oracle.c"),
                os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm"], exe, tmp_path)
    assert "oracle driver" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ needed")
def test_host_abi_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_san")
    out = _run(["g++", *SAN, "-std=c++17", "-ffp-contract=off", '-DDZS_SOURCE_HASH="sanitize"',
                "-I", os.path.join(ROOT, "include"), "-o", exe,
                os.path.join(ROOT, "paper_2005_05328_amd", "csrc", "cosmo.cpp"),
                os.path.join(ROOT, "tests", "sanitize", "host_abi_driver.cpp"), "-lm"], exe,
               tmp_path)
    assert "0 unexpected results" in out
