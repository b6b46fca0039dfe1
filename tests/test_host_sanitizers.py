"""The oracle and the plan builder's host code under AddressSanitizer and
UndefinedBehaviorSanitizer: both are rebuilt with gcc / g++ and the sanitizers,
driven at small sizes by the programs in tests/host/, and must run clean (any
report aborts the program).  The drivers also check properties fixed by the
mathematics (exact round trips of the sampling theorems; ring identities, GL
weights and the half-step shift spectra of the MW theta filter)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, exe, tmp_path):
    subprocess.check_call(cmd, cwd=ROOT)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    out = p.stdout + p.stderr
    if "does not come first in initial library list" in out:
        pytest.skip("the sanitizer runtime cannot be loaded first in this environment")
    assert p.returncode == 0, out[-4000:]
    assert "OK" in p.stdout
    assert "runtime error" not in out and "AddressSanitizer" not in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_san"
    _run(["gcc", *SAN, "-fopenmp", "oracle/s2oracle.c", "tests/host/oracle_san.c", "-lm", "-o", str(exe)], exe,
         tmp_path)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_plan_builder_under_sanitizers(tmp_path):
    exe = tmp_path / "consts_san"
    _run(["g++", *SAN, "-std=gnu++17", "-I", "paper_2311_14670_amd/csrc", "paper_2311_14670_amd/csrc/s2mi_consts.cpp",
          "tests/host/consts_san.cpp", "-lquadmath", "-o", str(exe)], exe, tmp_path)
