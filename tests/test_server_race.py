"""The serving runtime under concurrent clients, on the CPU (mock executor):
tests/server_stress.cpp drives submit / poll / release / statistics from
several threads and checks that every request completes exactly once within
the budget.  It runs against the library as built, and against a copy whose
server is built with ThreadSanitizer (host code only), which must report no
data race."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "include")
PKG = os.path.join(ROOT, "paper_2207_06803_amd")
SRC = os.path.join(ROOT, "tests", "server_stress.cpp")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    return r.returncode, r.stdout + r.stderr


def test_stress_against_the_library(tmp_path):
    exe = str(tmp_path / "stress")
    rc, out = _run(["g++", "-O1", "-std=c++17", "-pthread", "-I", INC, SRC, "-L", PKG, "-lfftc",
                    f"-Wl,-rpath,{PKG}", "-o", exe])
    assert rc == 0, out
    rc, out = _run([exe, "6", "2000"])
    assert rc == 0, out
    assert "bad 0" in out


def test_stress_under_thread_sanitizer(tmp_path):
    objs = sorted(glob.glob(os.path.join(ROOT, "_build", "obj", "*.o")))
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG) and objs):
        pytest.skip("needs hipcc, clang++ and the objects of a build (run __graft_entry__.build())")
    server_o = str(tmp_path / "server_tsan.o")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-x", "hip",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=thread",
           "-I", INC, "-c", os.path.join(PKG, "csrc", "server.cpp"), "-o", server_o]
    rc, out = _run(cmd)
    assert rc == 0, out
    lib = str(tmp_path / "libfftc_tsan.so")
    rest = [o for o in objs if not o.endswith("server.cpp.o")]
    rc, out = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=thread",
                    "-o", lib, *rest, server_o, "-lpthread"])
    assert rc == 0, out
    exe = str(tmp_path / "stress_tsan")
    rc, out = _run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=thread", "-I", INC, SRC, lib,
                    f"-Wl,-rpath,{tmp_path}", "-o", exe])
    assert rc == 0, out
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    rc, out = _run([exe, "4", "1000"], env=env)
    assert rc == 0 and "ThreadSanitizer" not in out, out
