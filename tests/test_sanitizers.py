"""The oracle (oracle.c) and the library's host build (forest_build.cpp)
under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU: small
drivers (tests/sanitize/) build and search plain, reflected and jittered
forests and check basic invariants; any sanitizer report fails the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=600, env=SAN_ENV)
    assert r.returncode == 0, f"{cmd[0]} exited {r.returncode}\n{r.stdout}\n{r.stderr}"
    return r.stdout


def test_oracle_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_check")
    _run([gcc, "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-ffp-contract=off", "-o", exe, os.path.join(HERE, "sanitize", "oracle_check.c"),
          os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-lpthread"], str(tmp_path))
    assert "passed" in _run([exe], str(tmp_path))


def test_host_forest_build_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "forest_check")
    # host code only: each -fsanitize applies to the host compilation
    _run([hipcc, "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
          "-fsanitize=undefined", "-fno-omit-frame-pointer", "-o", exe,
          os.path.join(HERE, "sanitize", "forest_check.cpp"),
          os.path.join(ROOT, "paper_1603_09596_amd", "csrc", "forest_build.cpp"), "-lpthread"],
         str(tmp_path))
    assert "passed" in _run([exe], str(tmp_path))
