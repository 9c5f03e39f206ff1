"""Build ``libmmpm.so`` (HIP kernels for gfx950 + host runtime + C ABI) with hipcc.

``python -m paper_2310_12441_amd.build`` compiles every source in ``csrc/``
and links them into ``paper_2310_12441_amd/lib/libmmpm.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "lib")
LIB = os.path.join(OUT_DIR, "libmmpm.so")
OBJ_DIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]
# Packed FP32 instructions stay off in every device object.
DEVICE = ["-x", "hip", "--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-fconstexpr-steps=20000000",  # the compile-time check of every LDS address of the 16-wave NTT
          "-munsafe-fp-atomics"]
HOST = ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


# Host AddressSanitizer (host code only: every sanitizer flag applies to the host
# pass; the gfx950 code objects are the same as in the plain build).
ASAN_DIR = os.path.join(HERE, "lib_asan")
ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def _compile(src: str, verbose: bool, obj_dir: str = OBJ_DIR, extra=()) -> str:
    obj = os.path.join(obj_dir, src + ".o")
    flags = DEVICE if src.endswith(".hip") else HOST
    cmd = [HIPCC] + flags + COMMON + list(extra) + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    os.makedirs(OUT_DIR, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


def build_asan(verbose: bool = False) -> str:
    """The library with host AddressSanitizer, ``lib_asan/libmmpm_asan.so``, and the
    C driver ``tests/c/abi_driver.c`` linked against it (``lib_asan/abi_driver``):
    the driver walks every entry point of the C ABI, so the host runtime's memory
    errors surface on a GPU run of it.  Not part of ``build()``."""
    obj_dir = os.path.join(ASAN_DIR, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, obj_dir, ASAN), srcs))
    lib = os.path.join(ASAN_DIR, "libmmpm_asan.so")
    steps = [
        [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC"] + ASAN + ["-o", lib] + objs + ["-lpthread"],
        [HIPCC, "-x", "c", "-O1", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROOT, "include"),
         "-I/opt/rocm/include"] + ASAN + [os.path.join(ROOT, "tests", "c", "abi_driver.c"), "-o",
                                          os.path.join(ASAN_DIR, "abi_driver"), "-L" + ASAN_DIR, "-lmmpm_asan",
                                          "-Wl,-rpath," + ASAN_DIR, "-L/opt/rocm/lib", "-lamdhip64",
                                          "-Wl,-rpath,/opt/rocm/lib", "-lm"],
    ]
    for cmd in steps:
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"asan build failed\n{res.stdout}\n{res.stderr}")
    return lib


if __name__ == "__main__":
    if "--asan" in sys.argv:
        print(build_asan(verbose="-v" in sys.argv))
    else:
        build(verbose="-v" in sys.argv)
        print(LIB)
