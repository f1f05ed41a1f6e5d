"""Build libddfem.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libddfem.so")
SOURCES = [os.path.join(HERE, "csrc", "ddfem.hip"), os.path.join(HERE, "csrc", "plan.cpp")]
HEADERS = [os.path.join(HERE, "csrc", "kernels.hpp"), os.path.join(HERE, "csrc", "pic.hpp"),
           os.path.join(HERE, "csrc", "mixed.hpp"), os.path.join(HERE, "csrc", "dp2.hpp"),
           os.path.join(HERE, "csrc", "plan.hpp"),
           os.path.join(ROOT, "include", "ddfem.h")]

FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *FLAGS, "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc"),
           *SOURCES, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libddfem.so")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
