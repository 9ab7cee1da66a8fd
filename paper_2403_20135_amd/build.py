"""Build the gfx950 shared library libsdc_mi355x.so in-tree with hipcc (no GPU needed)."""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libsdc_mi355x.so")
SOURCES = ["api.cpp", "setup.hip", "legendre.hip", "grid.hip", "update.hip", "adjoint.hip", "imex2.hip",
           "coriolis.hip"]
ARCH = "gfx950"
LINK_LIBS = ["-lroctx64"]             # roctx phase ranges (SDC_ROCTX)


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the HIP library)")


def compile_flags():
    return [f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall",
            "-Wno-unused-function", "-Wno-unused-command-line-argument",
            # no packed FP32 instructions in any device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # MFMA accumulators in ordinary VGPRs (no AGPR copies around every MFMA in loops)
            "-mllvm", "-amdgpu-mfma-vgpr-form",
            f"-I{os.path.join(ROOT, 'include')}"]


def _compile(src: str, extra) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), "-x", "hip", *compile_flags(), *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, extra=()) -> str:
    """Compile every source and link the shared library; returns its path.  Always rebuilds."""
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, list(extra)), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, *LINK_LIBS]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer"]


def build_host_sanitized() -> str:
    """The library with AddressSanitizer and UndefinedBehaviorSanitizer on the host code of the C
    ABI (argument validation, handle bookkeeping; device code unchanged) for CPU-side checks of
    the host paths.  Returns the path of _build/asan/libsdc_asan.so; load it in a process that
    preloads the sanitizer runtime (sanitizer_runtime())."""
    out_dir = os.path.join(BUILD, "asan")
    os.makedirs(out_dir, exist_ok=True)

    def one(src):
        if src == "api.cpp":
            obj = os.path.join(out_dir, "api.o")
            cmd = [hipcc(), "-x", "hip", *compile_flags(), "-O1", "-g", *HOST_SANITIZE, "-c",
                   os.path.join(CSRC, src), "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
            return obj
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        return obj if os.path.exists(obj) else _compile(src, [])

    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(one, SOURCES))
    lib = os.path.join(out_dir, "libsdc_asan.so")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *HOST_SANITIZE, "-o", lib, *objs, *LINK_LIBS]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    return lib


def sanitizer_runtime() -> str:
    """Path of the host AddressSanitizer runtime of the ROCm clang (to preload)."""
    import glob
    cands = sorted(glob.glob(os.path.join(os.path.dirname(os.path.dirname(hipcc())), "lib", "llvm", "lib",
                                          "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so")))
    if not cands:
        raise RuntimeError("libclang_rt.asan-x86_64.so not found")
    return cands[-1]


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
