"""Build ``libsf.so`` (the HIP C-ABI library) for gfx950 with hipcc.

Every .hip file under csrc/ is compiled separately (in parallel) and linked
into one shared library next to this file.  Packed FP32 instructions are
disabled (-packed-fp32-ops).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsf.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("SF_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I" + os.path.join(os.path.dirname(HERE), "include"),
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function"]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


# AddressSanitizer on the host half only (device code is never instrumented)
HOST_ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
ASAN_LIB = os.path.join(HERE, "libsf_asan.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile libsf.so; sanitize=True builds libsf_asan.so, whose host code
    carries AddressSanitizer checks (load it with clang's ASan runtime
    preloaded; the CPU-side tests use it)."""
    bdir = BUILD + ("_asan" if sanitize else "")
    lib_out = ASAN_LIB if sanitize else LIB
    extra = HOST_ASAN if sanitize else []
    os.makedirs(bdir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    cc = hipcc()

    def compile_one(src):
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        cmd = [cc, *FLAGS, *extra, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr)
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = lib_out + ".tmp"
    cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *extra, "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib_out)
    return lib_out


def asan_runtime() -> str:
    """clang's AddressSanitizer runtime matching hipcc (to preload)."""
    for d in sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux"), reverse=True):
        p = os.path.join(d, "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    raise RuntimeError("clang AddressSanitizer runtime not found")


if __name__ == "__main__":
    print(build(verbose=True))
