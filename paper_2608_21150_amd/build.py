"""Build libdycore.so (HIP for gfx950 + host C++) in the package directory.

Usage: python -m paper_2608_21150_amd.build   (always recompiles)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libdycore.so")
BUILD = os.path.join(PKG, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]
# host grid layer: no FP contraction so floating-point decisions are taken as written
CXX_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-Wall", "-ffp-contract=off", "-I", INCLUDE, "-I", CSRC]

# per-source extra flags: the network kernels keep MFMA results in ordinary
# VGPRs (no accumulator-register copies before the activations read them)
EXTRA_FLAGS = {"mlp.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}

SOURCES = [
    ("grid.cpp", "cxx"),
    ("abi.hip", "hip"),
    ("kernels.hip", "hip"),
    ("ensemble.hip", "hip"),
    ("mlp.hip", "hip"),
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for name, kind in SOURCES:
        src = os.path.join(CSRC, name)
        if not os.path.exists(src):
            continue
        obj = os.path.join(BUILD, name + ".o")
        if kind == "hip":
            cmd = [HIPCC, *HIP_FLAGS, *EXTRA_FLAGS.get(name, []), "-c", src, "-o", obj]
        else:
            cmd = [shutil.which("g++") or "g++", *CXX_FLAGS, "-c", src, "-o", obj]
        jobs.append((cmd, obj))
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(lambda j: _run(j[0]), jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *[o for _, o in jobs], "-o", tmp])
    os.replace(tmp, LIB)
    build_c_driver()
    return LIB


def build_c_driver() -> str:
    """The plain-C host driver (examples/c_driver.c): links the library and
    the system HIP runtime, finds libdycore.so next to the package."""
    src = os.path.join(PKG, "examples", "c_driver.c")
    out = os.path.join(PKG, "examples", "c_driver")
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    cc = shutil.which("gcc") or "gcc"
    tmp = out + ".tmp"
    _run([cc, "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", INCLUDE, "-I", os.path.join(rocm, "include"),
          src, "-o", tmp, "-L", PKG, "-ldycore", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
          "-Wl,-rpath,$ORIGIN/..", "-Wl,-rpath," + os.path.join(rocm, "lib")])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
