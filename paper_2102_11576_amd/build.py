"""Build librsfde.so for gfx950 in-tree with hipcc.

Every HIP translation unit is compiled with packed-FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops); the host warns that it
does not know the feature, which is harmless.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librsfde.so")

SOURCES = ["kernels_mv.hip", "pc_f64.hip", "pc_f32.hip", "pc_chirp_f64.hip", "pc_chirp_f32.hip",
           "kernels_krylov.hip", "krylov_dot.hip", "krylov_axpy.hip", "krylov_update.hip",
           "krylov_block.hip", "gemm_bf16.hip", "noalloc.hip", "rsfde_host.cpp"]
ARCH = os.environ.get("RSFDE_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _flags():
    return ["-std=c++17", "-O3", f"--offload-arch={ARCH}", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + _flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = True) -> str:
    """Compile every source and link librsfde.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def build_selftest() -> str:
    """Host-only self-test of the FFT index arithmetic (g++, no GPU)."""
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "fft_selftest")
    cmd = ["g++", "-std=c++17", "-O2", "-o", exe, os.path.join(CSRC, "fft_selftest.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr)
    return exe


# Host-only sanitizers: each -fsanitize= on a hipcc line follows -Xarch_host, so
# the device code is built as usual.  The shared library expects the clang
# AddressSanitizer runtime to be preloaded (asan_runtime()).
_SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    """Path of the clang AddressSanitizer runtime that the sanitised library links against."""
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang++"
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("clang AddressSanitizer runtime not found")
    return path


def build_sanitized() -> tuple[str, str]:
    """CPU build with AddressSanitizer and UndefinedBehaviorSanitizer on the host
    code: the plan set-up, validation and solver loop (rsfde_host.cpp) linked
    with the device objects of build() into _build/librsfde_asan.so, and the
    FFT engine self-test built by g++ with both sanitizers.  Returns (library,
    self-test executable)."""
    os.makedirs(BUILD, exist_ok=True)
    newest = max(os.path.getmtime(os.path.join(CSRC, f)) for f in os.listdir(CSRC))
    objs = []
    for src in SOURCES:
        if src == "rsfde_host.cpp":
            continue
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        if not os.path.exists(obj) or os.path.getmtime(obj) < newest:  # any source or header newer
            obj = _compile(src)
        objs.append(obj)
    host = os.path.join(BUILD, "rsfde_host_asan.o")
    cmd = [hipcc()] + _flags() + _SAN_HOST + ["-g", "-c", os.path.join(CSRC, "rsfde_host.cpp"), "-o", host]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc (sanitised host) failed:\n{r.stderr[-6000:]}")
    lib = os.path.join(BUILD, "librsfde_asan.so")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-shared-libasan"] + _SAN_HOST + \
        ["-o", lib, host] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link (sanitised) failed:\n{r.stderr[-6000:]}")
    exe = os.path.join(BUILD, "fft_selftest_asan")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-o", exe, os.path.join(CSRC, "fft_selftest.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr)
    return lib, exe


if __name__ == "__main__":
    build()
    sys.exit(0)
