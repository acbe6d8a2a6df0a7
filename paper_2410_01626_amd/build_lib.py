"""Build the HIP library libfmmcph.so for gfx950 (in-tree, next to this file)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfmmcph.so")
SOURCES = [os.path.join(CSRC, "fmm_api.hip"), os.path.join(CSRC, "lambda_dynamics.hip"),
           os.path.join(CSRC, "operators.cpp")]
HEADERS = [os.path.join(CSRC, f) for f in ("fmm_kernels.hip", "exclusions.hip", "fmm_internal.h",
                                           "operators.h")] + [
    os.path.join(ROOT, "include", "fmmcph.h")]


def hipcc_cmd(out: str, arch: str = "gfx950") -> list[str]:
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    return [hipcc, "--offload-arch=" + arch, "-O3", "-std=c++17", "-fPIC", "-shared",
            # no packed-FP32 instructions anywhere in device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
            *SOURCES, "-o", out]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = hipcc_cmd(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
