"""Build the C-ABI library libcsv.so (HIP, gfx950) in the package folder."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", f) for f in ("csv_decode.hip", "csv_encode.cpp")]
LIB = os.path.join(HERE, "libcsv.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # packed fp32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-pthread"]


def build() -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC] + FLAGS + SRC + ["-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
