"""Build the gfx950 shared library libkpm.so in-tree with hipcc.

    python -m paper_2104_13218_amd.build
    python -m paper_2104_13218_amd.build --sanitize

Packed-FP32 instructions are disabled for all HIP code (their generated
forms are not trusted on the target machines); everything else is -O3.

--sanitize builds libkpm_asan.so: the same sources with the host code (the
C ABI, planner and launch layer) instrumented by AddressSanitizer and
UndefinedBehaviorSanitizer; device code is compiled as usual.  It is loaded
with the sanitizer runtime preloaded (see tests/test_abi_sanitized.py).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libkpm.so")
LIB_ASAN = os.path.join(HERE, "libkpm_asan.so")
SOURCES = ["kpm_kernels.hip", "kpm_slice.hip", "kpm_thermo.hip", "kpm_adjoint.hip", "kpm_ftlm.hip", "kpm_ed.hip",
           "kpm_api.hip"]
ARCH = os.environ.get("KPM_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def common_flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", CSRC]


# host-side instrumentation only (each sanitizer flag applies to the host pass)
SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer",
            "-Xarch_host", "-fsanitize=address",
            "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined"]


def sanitizer_runtime() -> str:
    """The AddressSanitizer runtime of the ROCm clang (to preload)."""
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "lib", "llvm", "bin", "clang")
    for c in (clang, "/opt/rocm/llvm/bin/clang"):
        if os.path.exists(c):
            r = subprocess.run([c, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                               text=True)
            path = r.stdout.strip()
            if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path):
                return path
    raise RuntimeError("AddressSanitizer runtime not found")


def _compile(src: str, build_dir: str, extra=()) -> str:
    obj = os.path.join(build_dir, src.replace(".hip", ".o"))
    cmd = [hipcc(), *common_flags(), *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    build_dir = os.path.join(HERE, "_build_asan" if sanitize else "_build")
    lib = LIB_ASAN if sanitize else LIB
    os.makedirs(build_dir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    extra = SANITIZE if sanitize else ()
    with ThreadPoolExecutor(max_workers=min(4, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir, extra), srcs))
    tmp = lib + ".tmp"
    # the sanitized library leaves the runtime's symbols to the preloaded runtime
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
