"""Host code under sanitizers (CPU only): the library's host-only sources
(CSR loading, validation, binarization, features) and the CPU oracle are
built with AddressSanitizer + UndefinedBehaviorSanitizer, and the oracle
(which runs thread pools) also with ThreadSanitizer, then driven on valid
and malformed inputs.  Any sanitizer report fails the build's run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2210_16998_amd", "csrc")
SAN = os.path.join(ROOT, "tests", "sanitize")
ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
HIP_HOST = ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]


def _build_and_run(tmp_path, name, srcs, flags, extra=()):
    exe = str(tmp_path / name)
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-pthread"] + list(flags) + list(extra) + srcs + \
        ["-o", exe]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_library_under_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "host_lib", [os.path.join(SAN, "host_lib_driver.cpp"),
                                                os.path.join(CSRC, "graph.cpp"),
                                                os.path.join(CSRC, "features.cpp")],
                         ASAN, HIP_HOST)
    assert "loads ok" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "oracle_asan", [os.path.join(SAN, "oracle_driver.cpp"),
                                                   os.path.join(ROOT, "oracle", "oracle.cpp")],
                         ASAN)
    assert "oracle driver ok" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_tsan(tmp_path):
    out = _build_and_run(tmp_path, "oracle_tsan", [os.path.join(SAN, "oracle_driver.cpp"),
                                                   os.path.join(ROOT, "oracle", "oracle.cpp")],
                         ["-fsanitize=thread"])
    assert "oracle driver ok" in out
