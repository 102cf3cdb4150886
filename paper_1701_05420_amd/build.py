"""Compile the gfx950 library libcumulants.so in place (hipcc, no JIT)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcumulants.so")
SOURCES = ["kernels.hip", "api.cpp"]
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer (the device code
# is built as usual): a separate library for checking the host planner.
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-g", "-shared-libsan"]
SAN_LIB = os.path.join(HERE, "libcumulants.asan.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    lib = SAN_LIB if sanitize else LIB
    tmp = lib + ".tmp"
    cmd = [hipcc, *FLAGS, *(SANITIZE if sanitize else []), "-I", os.path.join(HERE, "..", "include"),
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    import sys

    print(build(verbose=True, sanitize="--sanitize" in sys.argv[1:]))
