"""Build libwmc.so in-tree for gfx950.

    python -m paper_2006_15512_amd.build              # libwmc.so
    python -m paper_2006_15512_amd.build --sanitize   # + _build/san/libwmc.so

The host planner (C++17) is compiled with g++, the kernels with hipcc for
gfx950 only; packed-FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libwmc.so")
BUILD_DIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

HOST_SOURCES = ["wmc_host.cpp"]
DEVICE_SOURCES = ["wmc_device.hip", "wmc_batch.hip", "wmc_serve.hip"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


SAN_DIR = os.path.join(BUILD_DIR, "san")
SAN_LIB = os.path.join(SAN_DIR, "libwmc.so")


def build_sanitized(verbose: bool = False) -> str:
    """The host planner (wmc_host.cpp) under AddressSanitizer and
    UndefinedBehaviorSanitizer, linked with the ordinary device objects into
    _build/san/libwmc.so (a CPU build for the planner tests: run them with
    WMC_LIBRARY pointing at it and the sanitizer runtime preloaded).  The
    device code is not instrumented."""
    build(verbose)
    os.makedirs(SAN_DIR, exist_ok=True)
    inc = ["-I", CSRC, "-I", os.path.join(ROOT, "include")]
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
    host_o = os.path.join(SAN_DIR, "wmc_host.cpp.o")
    _run(["g++", "-std=c++17", "-O1", "-g", *san, "-fPIC", *inc, "-c", os.path.join(CSRC, "wmc_host.cpp"),
          "-o", host_o], verbose)
    dev_o = [os.path.join(BUILD_DIR, s + ".o") for s in DEVICE_SOURCES]
    rocm = os.path.dirname(os.path.dirname(HIPCC))
    _run(["g++", "-shared", *san, host_o, *dev_o, "-L", os.path.join(rocm, "lib"), "-lamdhip64",
          "-Wl,-rpath," + os.path.join(rocm, "lib"), "-o", SAN_LIB], verbose)
    return SAN_LIB


def build(verbose: bool = False, debug: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    inc = ["-I", CSRC, "-I", os.path.join(ROOT, "include")]
    opt = ["-O0", "-g"] if debug else ["-O3"]
    objs, cmds = [], []
    for s in HOST_SOURCES:
        o = os.path.join(BUILD_DIR, s + ".o")
        cmds.append(["g++", "-std=c++17", *opt, "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter", *inc, "-c",
                     os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in DEVICE_SOURCES:
        o = os.path.join(BUILD_DIR, s + ".o")
        cmds.append([HIPCC, "-std=c++17", *opt, "-fPIC", f"--offload-arch={ARCH}", *DEVICE_FLAGS, "-Wall",
                     "-Wno-unused-command-line-argument", *inc, "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    # the translation units are independent: compile them side by side
    procs = []
    for c in cmds:
        if verbose:
            print(" ".join(c), flush=True)
        procs.append(subprocess.Popen(c))
    failed = [c for c, p in zip(cmds, procs) if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv, debug="--debug" in sys.argv))
