"""Build the HIP library libsflow.so in-tree for gfx950 with hipcc.

Usage: python -m paper_2406_18031_amd.build  (or build() from Python).
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libsflow.so")
SOURCES = [os.path.join(PKG, "csrc", f) for f in ("sflow_kernels.hip", "sflow_cnn.hip",
                                                         "sflow_abi.hip", "sflow_net.hip",
                                                         "sflow_copy.hip", "sflow_stereo.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -packed-fp32-ops: no packed FP32 instructions in device code; -ffp-contract=off: only the
# FMAs written out (fmaf) are fused, so every code path rounds alike
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument",
         "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]


# Host-side undefined-behaviour checks for a check build: every check compiles to a trap
# instruction in the host code (no sanitizer runtime to load, so the library still loads into
# an ordinary Python process); device code is built as in the product library.
UBSAN_FLAGS = ["-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fsanitize-trap=undefined",
               "-Xarch_host", "-fno-sanitize-recover=all"]
LIB_UBSAN = os.path.join(PKG, "libsflow_ubsan.so")


def build(verbose: bool = False, ubsan: bool = False) -> str:
    """Build libsflow.so; with ubsan=True the host-UB-trapping check build libsflow_ubsan.so
    (loaded instead of the product library when SFLOW_LIB names it)."""
    lib = LIB_UBSAN if ubsan else LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, *FLAGS, *(UBSAN_FLAGS if ubsan else []), *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed building {os.path.basename(lib)}")
    if verbose and r.stderr.strip():
        sys.stderr.write(r.stderr)
    os.replace(tmp, lib)
    return lib


ASAN_DRIVER_SRC = os.path.join(ROOT, "tests", "host_asan", "abi_asan_driver.hip")
ASAN_DRIVER = os.path.join(ROOT, "tests", "host_asan", "abi_asan_driver")


def build_asan_driver(verbose: bool = False) -> str:
    """The C ABI driver of tests/host_asan, built with the library's sources into one executable
    whose host code runs under AddressSanitizer (its runtime linked in); device code as in the
    product library."""
    flags = [f for f in FLAGS if f not in ("-fPIC", "-shared")]
    cmd = [HIPCC, *flags, "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
           "-fno-omit-frame-pointer", *SOURCES, ASAN_DRIVER_SRC, "-o", ASAN_DRIVER]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building the ABI driver")
    return ASAN_DRIVER


if __name__ == "__main__":
    if "--asan" in sys.argv:
        print(build_asan_driver(verbose=True))
    else:
        print(build(verbose=True, ubsan="--ubsan" in sys.argv))
