"""Host-side checks of the library (CPU).

The partition tree and admissibility lists run under AddressSanitizer and
UndefinedBehaviorSanitizer, checked for structure by tests/host/tree_check.cpp
over several sizes and leaf sizes; only the host pass is instrumented (each
-fsanitize follows -Xarch_host).  tests/host/abi_c_check.c is a plain C99
client of include/spdhss.h, linked against the library."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_tree_under_asan_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "tree_check")
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2011_07632_amd", "csrc"),
           os.path.join(ROOT, "tests", "host", "tree_check.cpp"),
           os.path.join(ROOT, "paper_2011_07632_amd", "csrc", "tree.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "tree_check ok" in r.stdout, (r.stdout + r.stderr)[-3000:]


def test_plain_c_client(tmp_path):
    """include/spdhss.h is C99 and the library links and answers from C."""
    lib_dir = os.path.join(ROOT, "paper_2011_07632_amd")
    if not os.path.exists(os.path.join(lib_dir, "libspdhss.so")):
        pytest.skip("library not built")
    exe = str(tmp_path / "abi_c_check")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host", "abi_c_check.c"),
           "-L", lib_dir, "-lspdhss", f"-Wl,-rpath,{lib_dir}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "abi_c_check ok" in r.stdout, (r.stdout + r.stderr)[-3000:]
