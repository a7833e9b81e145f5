"""Build libbssmppi.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc.

Every translation unit is compiled to an object of its own in parallel (the solve kernel is
split by particles-per-lane count into four units), then the objects are linked.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libbssmppi.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = [os.path.join(HERE, "csrc", f)
           for f in ("bss_solve_pm.hip", "bss_solve_p8.hip", "bss_solve_p4.hip", "bss_solve_p2.hip",
                     "bss_solve_p1.hip", "bss_solve8.hip", "bss_kernels.hip", "bss_noalloc.hip",
                     "bss_api.cpp",
                     "bss_server.cpp")]

# gfx950 only; packed-FP32 instructions are disabled (the compiler must not form v_pk_* FP32
# ops); no fast-math: the kernels rely on IEEE single/double semantics.
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def _compile(src, extra, verbose):
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = ["hipcc"] + FLAGS + list(extra) + ["-c", "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, cwd="/tmp", capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, extra=None) -> str:
    extra = list(extra or [])
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as pool:
        objs = list(pool.map(lambda s: _compile(s, extra, verbose), SOURCES))
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd="/tmp")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
