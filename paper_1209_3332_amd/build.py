"""Build librecon.so (HIP, gfx950) in-tree with hipcc.

Usage: ``python paper_1209_3332_amd/build.py`` (run as a script: importing the
package first would load the library this builds).
The library lands next to this file so that it travels with the source tree.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "recon.hip")
# host-only translation units: the tile-pipeline scheduler and its CPU variants
HOST_SRCS = [os.path.join(HERE, "csrc", f) for f in ("pipeline.cpp", "host_ops.cpp")]
LIB = os.path.join(HERE, "librecon.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    """Compile csrc/recon.hip and the host sources into librecon.so (always recompiles)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-o", tmp, SRC] + HOST_SRCS
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
