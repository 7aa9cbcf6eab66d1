"""Host code under AddressSanitizer and UBSan (CPU only): the oracle's C and the
library's host table builder, each linked into a small driver
(tests/native/) that calls every entry point on small inputs.  The run must end
with status 0 and report no sanitizer finding."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _build_and_run(tmp_path, cmd, exe):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitizer" in (r.stderr + r.stdout).lower() and "cannot find" in r.stderr.lower():
        pytest.skip("sanitizer runtime not available")
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    env.pop("LD_PRELOAD", None)
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = run.stdout + run.stderr
    assert run.returncode == 0, out
    assert "runtime error" not in out and "ERROR: AddressSanitizer" not in out, out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", *SAN, "-fopenmp", "-o", exe, os.path.join(NATIVE, "oracle_sanitize.c"),
           os.path.join(ROOT, "oracle", "soap_oracle.c"), "-lm"]
    _build_and_run(tmp_path, cmd, exe)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_host_tables_under_sanitizers(tmp_path):
    exe = str(tmp_path / "tables_sanitize")
    cmd = ["g++", *SAN, "-std=gnu++17", "-o", exe, os.path.join(NATIVE, "tables_sanitize.cpp"),
           os.path.join(ROOT, "paper_1905_02142_amd", "csrc", "tables.cpp"), "-lquadmath"]
    _build_and_run(tmp_path, cmd, exe)
