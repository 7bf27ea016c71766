"""The FP64 oracle (C) and the library's host code (argument validation,
tiles, the tuning cache, the exact host pair counter) under AddressSanitizer
and UndefinedBehaviorSanitizer, on the CPU: sanitizer builds of both, and the
CPU tests that drive them run in a child process with clang's sanitizer
runtime preloaded; any report fails the run.  A snippet with a heap overflow,
built and run the same way, first shows that the sanitizers are live.  Device
code is not instrumented (no GPU sanitizer is used)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

OVERFLOW = r"""
#include <stdlib.h>
int write_past_end(int n) { int* a = (int*)malloc(sizeof(int) * n); a[n] = 1; int r = a[0]; free(a); return r; }
"""


def _env(tmp_path, rt, lib=None, olib=None):
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    if lib:
        env["KM_LIBRARY"] = lib
    if olib:
        env["KM_ORACLE_LIBRARY"] = olib
    return env


def test_host_code_and_oracle_under_asan_ubsan(tmp_path):
    from paper_1204_1225_amd import build

    import oracle

    try:
        rt = build.asan_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    # the sanitizers are live: an overflow built with the same flags is reported
    src = tmp_path / "overflow.c"
    src.write_text(OVERFLOW)
    so = str(tmp_path / "liboverflow.so")
    subprocess.run(["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-fsanitize=address,undefined", "-shared-libasan",
                    "-shared", "-fPIC", str(src), "-o", so], check=True)
    r = subprocess.run([sys.executable, "-c", f"import ctypes; ctypes.CDLL({so!r}).write_past_end(4)"],
                       env=_env(tmp_path, rt), capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr

    lib = build.build_sanitized(str(tmp_path / "libkirchhoff_asan.so"))
    olib = oracle.build_sanitized(str(tmp_path / "liboracle_asan.so"))
    tests = ["tests/test_abi.py", "tests/test_count_host.py", "tests/test_oracle_pins.py",
             "tests/test_oracle_table.py", "tests/test_oracle_aa.py"]
    check = ("import sys; sys.path.insert(0, {root!r})\n"
             "from paper_1204_1225_amd import _lib\nimport oracle\n"
             "assert _lib.LIB_PATH == {lib!r} and oracle._LIB == {olib!r}\n"
             "import ctypes; assert hasattr(ctypes.CDLL(None), '__asan_init')\n").format(root=ROOT, lib=lib, olib=olib)
    r = subprocess.run([sys.executable, "-c", check], env=_env(tmp_path, rt, lib, olib), capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([sys.executable, "-m", "pytest", *tests, "-q", "-p", "no:cacheprovider", "-m", "not gpu"],
                       env=_env(tmp_path, rt, lib, olib), capture_output=True, text=True, timeout=900, cwd=ROOT)
    out = r.stdout + r.stderr
    print(out[-600:])
    assert r.returncode == 0, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out
