"""Host code under AddressSanitizer, UndefinedBehaviorSanitizer and LeakSanitizer (CPU only):
the FP64 oracle driven through small solves of every reading, and the host side of the C ABI
(validation, allocation failures, NULL handles, the scratch check of the solve that allocates
nothing, server and batch argument checks).  The GPU kernels are not instrumented: the sanitizer
flags apply to host code only."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2408_00494_amd", "csrc")
LIBDIR = os.path.join(ROOT, "paper_2408_00494_amd")
ROCM_CLANG = "/opt/rocm/llvm/bin"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_asan")
        _run(["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
              "-I", os.path.join(ROOT, "oracle"), "-o", exe,
              os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "bss_oracle.c"),
              os.path.join(ROOT, "oracle", "bss_oracle8.c"), "-lm", "-lpthread"], tmp)
        r = _run([exe], tmp)
        assert "oracle driver: ok" in r.stdout


@pytest.mark.skipif(shutil.which("hipcc") is None or not os.path.exists(
    os.path.join(ROCM_CLANG, "clang++")), reason="needs hipcc and ROCm's clang")
@pytest.mark.skipif(not os.path.exists(os.path.join(LIBDIR, "libbssmppi.so")),
                    reason="libbssmppi.so not built")
def test_abi_host_code_under_asan_and_ubsan():
    """The ABI's host translation units are rebuilt with the host sanitizers and linked into a
    driver ahead of the library (which supplies the kernel launchers), so every call the driver
    makes runs instrumented code."""
    with tempfile.TemporaryDirectory() as tmp:
        host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-omit-frame-pointer"]
        common = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                  "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                  "-I", os.path.join(ROOT, "include")]
        objs = []
        procs = []
        for src in ("bss_api.cpp", "bss_server.cpp", "bss_noalloc.hip"):
            obj = os.path.join(tmp, src + ".o")
            objs.append(obj)
            procs.append(subprocess.Popen(["hipcc"] + common + host_san +
                                          ["-c", "-o", obj, os.path.join(CSRC, src)], cwd=tmp,
                                          stdout=subprocess.PIPE, stderr=subprocess.PIPE))
        for pr in procs:
            out, err = pr.communicate(timeout=600)
            assert pr.returncode == 0, err.decode()[-3000:]
        drv = os.path.join(tmp, "driver.o")
        _run([os.path.join(ROCM_CLANG, "clang"), "-O1", "-g", "-fsanitize=address,undefined",
              "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-c", "-o", drv,
              os.path.join(HERE, "abi_driver.c")], tmp)
        exe = os.path.join(tmp, "abi_asan")
        _run([os.path.join(ROCM_CLANG, "clang++"), "-fsanitize=address,undefined", "-o", exe,
              drv] + objs + ["-L", LIBDIR, "-l:libbssmppi.so", "-Wl,-rpath," + LIBDIR,
                             "-L", "/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"],
             tmp)
        r = _run([exe], tmp)
        assert "abi driver: ok" in r.stdout
