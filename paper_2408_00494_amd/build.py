"""Build libbssmppi.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libbssmppi.so")
SOURCES = [os.path.join(HERE, "csrc", f)
           for f in ("bss_kernels.hip", "bss_api.cpp", "bss_server.cpp")]

# gfx950 only; packed-FP32 instructions are disabled (the compiler must not form v_pk_* FP32
# ops); no fast-math: the kernels rely on IEEE single/double semantics.
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, extra=None) -> str:
    cmd = ["hipcc"] + FLAGS + list(extra or []) + ["-o", LIB + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd="/tmp")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
