"""Builds the HIP library ``libtdct.so`` (gfx950) in-tree with hipcc.

Every HIP code object is compiled for gfx950 only, with packed-FP32
instruction selection disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libtdct.so")
HOSTCHECK_SRC = os.path.join(ROOT, "tests", "hostcheck.cpp")
HOSTCHECK_LIB = os.path.join(ROOT, "tests", "libhostcheck.so")

SOURCES = ["tdct_kernels.hip", "tdct_probe.hip", "tdct_resident.hip", "tdct_static.hip",
           "tdct_batch.cpp", "tdct_server.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I" + INCLUDE, "-I" + CSRC]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# The resident kernel's atomics take a lane-0-only operand; a DPP scan folds
# them into one atomic per wave in a few dozen instructions.
PER_SOURCE = {"tdct_resident.hip": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=DPP"]}


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), out))
    if verbose and out.strip():
        print(out)


def build_lib(verbose: bool = False) -> str:
    objs = []
    bdir = os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(bdir, src + ".o")
        # hipcc compiles .cpp files as HIP too: every source names the target,
        # so no code object for any other GPU is made
        lang = ["-x", "hip"] + DEVICE
        _run([HIPCC] + COMMON + lang + PER_SOURCE.get(src, []) + ["-c", path, "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs +
         ["-lpthread"], verbose)
    os.replace(tmp, LIB)
    return LIB


def build_hostcheck(verbose: bool = False) -> str:
    """Host-only test helper built from the library's device header."""
    tmp = HOSTCHECK_LIB + ".tmp%d" % os.getpid()
    _run([HIPCC] + COMMON + ["-x", "hip"] + DEVICE + ["-shared", "-o", tmp, HOSTCHECK_SRC], verbose)
    os.replace(tmp, HOSTCHECK_LIB)
    return HOSTCHECK_LIB


def build(verbose: bool = False) -> str:
    lib = build_lib(verbose)
    build_hostcheck(verbose)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
