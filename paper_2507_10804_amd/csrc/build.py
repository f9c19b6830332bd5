"""Build the gfx950 shared library ``libfwi_mi355x.so`` next to the package.

hipcc cross-compiles for gfx950 without a GPU present.  Packed FP32 vector
instructions are disabled for every HIP translation unit, and implicit FMA
contraction is off: kernels state their FMAs explicitly so that every kernel
evaluates the leapfrog update in the same order.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libfwi_mi355x.so")
SOURCES = ["fwi_kernels.hip", "fwi_psf.hip", "fwi_lowrank.hip", "fwi_symbol.hip", "fwi_opt.hip",
           "fwi_calib.hip", "fwi_noalloc.hip", "fwi_api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build of the plan
# code (CPU checks only; the device code is built as usual).  Every sanitizer
# flag applies to the host pass alone.
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-shared-libasan"]
SANITIZED_LIB = os.path.join(HERE, "_build", "asan", "libfwi_mi355x.so")
EXAMPLE = os.path.join(PKG, "fwi_example")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source and link the library; with `sanitize`, the host
    plan code (fwi_api.cpp) carries ASan and UBSan and the library goes to
    _build/asan/ (load it with libclang_rt.asan preloaded)."""
    objs = []
    bdir = os.path.join(HERE, "_build", "asan") if sanitize else os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        extra = SANITIZE + ["-g"] if sanitize and src.endswith(".cpp") else []
        cmd = [HIPCC, *FLAGS, *extra, *lang, "-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    lib = SANITIZED_LIB if sanitize else LIB
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *(SANITIZE if sanitize else []),
           *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    if not sanitize:
        build_example(verbose)
    return lib


def build_example(verbose: bool = False) -> str:
    """Compile fwi_example.cpp, a host program (no device code) that calls the
    library through include/fwi.h and the HIP runtime API alone, and link it
    against the in-tree library (found next to the executable at run time)."""
    tmp = EXAMPLE + ".tmp%d" % os.getpid()
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    cmd = [os.environ.get("CXX", "g++"), "-O2", "-std=c++17", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(rocm, "include"),
           os.path.join(HERE, "fwi_example.cpp"), "-L", PKG, "-lfwi_mi355x",
           "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath,$ORIGIN",
           "-Wl,-rpath," + os.path.join(rocm, "lib"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, EXAMPLE)
    return EXAMPLE


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
