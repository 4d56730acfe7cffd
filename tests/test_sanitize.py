"""CPU builds of the host code under sanitizers: the library's graph-store
builder (multithreaded C++) and the oracle (C), driven by
tests/sanitize/host_check.cpp on seeded random graphs, once with the
address and undefined-behaviour sanitizers and once with the thread
sanitizer. The build is CPU-only (g++/gcc, no HIP code)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "tests", "sanitize", "host_check.cpp"),
       os.path.join(ROOT, "paper_2412_10287_amd", "csrc", "graph_build.cpp")]
ORACLE = os.path.join(ROOT, "oracle", "oracle.c")


def _build_and_run(tmp_path, flags):
    if not (shutil.which("g++") and shutil.which("gcc")):
        pytest.skip("no host C/C++ compiler")
    obj = str(tmp_path / "oracle.o")
    exe = str(tmp_path / "host_check")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", *flags, "-c", ORACLE, "-o", obj], check=True)
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", *flags, *SRC, obj, "-o", exe, "-lpthread"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.startswith("ok"), r.stdout
    return r.stdout


def test_host_code_asan_ubsan(tmp_path):
    print(_build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                                    "-fno-omit-frame-pointer"]))


def test_host_code_tsan(tmp_path):
    print(_build_and_run(tmp_path, ["-fsanitize=thread"]))
