"""Build the C-ABI library libcsv.so (HIP, gfx950) in the package folder."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", f) for f in ("csv_decode.hip", "csv_generic.hip", "csv_encode_gpu.hip", "csv_cache.hip", "csv_encode.cpp",
                                                   "csv_server.cpp")]
LIB = os.path.join(HERE, "libcsv.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # packed fp32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-pthread"]


def build(out: str = LIB, extra=()) -> str:
    """Compile the library; `extra` adds flags (e.g. -DCSV_PHASE_TIMING for
    the per-phase clock build)."""
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC] + FLAGS + list(extra) + SRC + ["-o", tmp])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
