"""Build libkirchhoff.so (HIP, gfx950) in-tree next to this file.

hipcc compiles every source under csrc/ as HIP for gfx950 with
-ffp-contract=off (the aperture decision and the migrate/demigrate pair
evaluation rely on unfused float32 arithmetic) and with packed-FP32
instruction selection disabled.  Objects go to _build/, the shared library
to paper_1204_1225_amd/libkirchhoff.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libkirchhoff.so")
SOURCES = ["km_api.cpp", "km_count.cpp", "km_migrate.hip", "km_demigrate.hip", "km_misc.hip", "km_cig.hip",
           "km_filter.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
        raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
    return obj


def build(verbose: bool = True) -> str:
    """Compile every HIP source and link libkirchhoff.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


# Host sources (no device code): the ones the sanitizer build instruments.
HOST_SOURCES = ["km_api.cpp", "km_count.cpp"]
SANITIZE_FLAGS = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    """clang's shared AddressSanitizer runtime (to preload into the process
    that loads a sanitizer build)."""
    import glob

    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise RuntimeError("clang's shared AddressSanitizer runtime is not installed")
    return found[-1]


def build_sanitized(out: str) -> str:
    """A build of the library whose host code (argument validation, tiles,
    the tuning cache, the host pair counter) carries AddressSanitizer and
    UndefinedBehaviorSanitizer checks; the device code is the normal one.  The
    sanitizer runtime is not linked in: load the library into a process that
    preloads asan_runtime()."""
    objs = [os.path.join(BUILD, os.path.splitext(f)[0] + ".o") for f in SOURCES if f not in HOST_SOURCES]
    if not all(os.path.exists(o) for o in objs):
        build(verbose=False)
    work = os.path.join(BUILD, "sanitize")
    os.makedirs(work, exist_ok=True)
    host_objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(work, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *[f for f in FLAGS if f != "-O3"], *SANITIZE_FLAGS, "-x", "hip", "-c",
               os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"sanitizer build of {src} failed:\n{r.stdout}{r.stderr}")
        host_objs.append(obj)
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *host_objs, *objs, "-o", out],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitizer link failed:\n{r.stdout}{r.stderr}")
    return out


if __name__ == "__main__":
    build()
    sys.exit(0)
