"""Build libfresco.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2305_15693_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfresco.so")
OBJDIR = os.path.join(ROOT, "_build")

SOURCES = ["plan.cpp", "spread.hip", "fft.hip", "lbfgs.hip", "pair.hip", "batch.hip", "type3.hip",
           "capi.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          "-I", OBJDIR, "-Wno-unused-command-line-argument"]


def _generate_tables() -> None:
    """Build and run csrc/gen_tables.cpp: writes _build/kernel_tables.h (the FP32
    kernel polynomials as compile-time constants)."""
    os.makedirs(OBJDIR, exist_ok=True)
    exe = os.path.join(OBJDIR, "gen_tables")
    cmd = [HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-D__HIP_PLATFORM_AMD__", os.path.join(CSRC, "gen_tables.cpp"),
           os.path.join(CSRC, "plan.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("table generator failed to build")
    out = os.path.join(OBJDIR, "kernel_tables.h")
    r = subprocess.run([exe, out + ".tmp"], capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("table generator failed")
    os.replace(out + ".tmp", out)


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer (device code is
# compiled as usual): the argument checks and host logic of the C ABI can run
# under the sanitizers on a machine without a GPU.
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _compile(src: str, objdir: str = OBJDIR, extra=()) -> str:
    os.makedirs(objdir, exist_ok=True)
    obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [HIPCC, "-c", "-x", "hip", *DEVICE_FLAGS, *COMMON, *extra, path, "-o", obj]
    else:
        cmd = [HIPCC, "-c", *COMMON, *extra, "-D__HIP_PLATFORM_AMD__", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"compile failed: {src}")
    return obj


def build(verbose: bool = False) -> str:
    _generate_tables()
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", *DEVICE_FLAGS, *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_host_sanitized(out_dir: str) -> str:
    """libfresco.so with host-side ASan + UBSan in out_dir (objects there too).
    Load it with the clang ASan runtime preloaded (host_sanitizer_runtime())."""
    _generate_tables()
    objdir = os.path.join(out_dir, "obj")
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, objdir, HOST_SANITIZE), SOURCES))
    lib = os.path.join(out_dir, "libfresco_hostsan.so")
    cmd = [HIPCC, "-shared", "-fPIC", *DEVICE_FLAGS, *HOST_SANITIZE, "-shared-libasan", *objs,
           "-o", lib]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    return lib


def host_sanitizer_runtime() -> str:
    """Path of the clang ASan runtime that a sanitized build needs preloaded."""
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True, check=True)
    return r.stdout.strip()


if __name__ == "__main__":
    build(verbose=True)
