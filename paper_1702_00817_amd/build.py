"""Builds the HIP library ``libtdct.so`` (gfx950) in-tree with hipcc.

Every HIP code object is compiled for gfx950 only, with packed-FP32
instruction selection disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libtdct.so")
HOSTCHECK_SRC = os.path.join(ROOT, "tests", "hostcheck.cpp")
HOSTCHECK_LIB = os.path.join(ROOT, "tests", "libhostcheck.so")

SOURCES = ["tdct_kernels.hip", "tdct_probe.hip", "tdct_resident.hip", "tdct_static.hip",
           "tdct_batch.cpp", "tdct_server.cpp", "tdct_tunecache.cpp", "tdct_host.cpp"]
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


def source_hash() -> str:
    """First 16 hex digits of the SHA-256 over the library's sources and
    header: built into the library, it keys the autotune cache, so shapes
    tuned for other kernel code are never taken."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".cpp", ".hpp")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    with open(os.path.join(INCLUDE, "tdct.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def _run_all(cmds, verbose):
    """Runs independent compile commands side by side (at most 4 at once)."""
    with ThreadPoolExecutor(max_workers=min(4, len(cmds))) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()


def build_lib(verbose: bool = False) -> str:
    objs, jobs = [], []
    bdir = os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    ident = ['-DTDCT_SOURCE_HASH="%s"' % source_hash()]
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(bdir, src + ".o")
        # hipcc compiles .cpp files as HIP too: every source names the target,
        # so no code object for any other GPU is made
        lang = ["-x", "hip"] + DEVICE
        jobs.append([HIPCC] + COMMON + ident + lang + PER_SOURCE.get(src, []) + ["-c", path, "-o", obj])
        objs.append(obj)
    _run_all(jobs, verbose)
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


# Host-only instrumentation: each -fsanitize= applies to the host pass alone
# (device code is never instrumented), so the sanitizer builds cover the
# C ABI's host logic -- validation, planning, the server's scheduler and its
# fake device -- and run on a machine without a GPU.
SANITIZE = {
    "address": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer"],
    "thread": ["-Xarch_host", "-fsanitize=thread"],
}
DRIVER_SRC = os.path.join(ROOT, "tests", "sanitize", "fake_device_driver.cpp")


def build_sanitized(kind: str, verbose: bool = False) -> str:
    """Builds the host part of the library's sources and the fake-device
    driver (tests/sanitize/fake_device_driver.cpp) into one executable
    instrumented by `kind` ("address": ASan + UBSan, "thread": TSan).
    Returns the executable's path (under _build/)."""
    flags = SANITIZE[kind]
    bdir = os.path.join(PKG, "_build", "sanitize_" + kind)
    os.makedirs(bdir, exist_ok=True)
    objs, jobs = [], []
    for src in SOURCES + [DRIVER_SRC]:
        path = src if os.path.isabs(src) else os.path.join(CSRC, src)
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        jobs.append([HIPCC] + COMMON + ["-O1", "-g", "-x", "hip"] + DEVICE + flags +
                    PER_SOURCE.get(src, []) + ["-c", path, "-o", obj])
        objs.append(obj)
    _run_all(jobs, verbose)
    exe = os.path.join(bdir, "fake_device_driver")
    _run([HIPCC, "--offload-arch=" + ARCH] + flags + ["-o", exe] + objs + ["-lpthread"], verbose)
    return exe


def build(verbose: bool = False) -> str:
    lib = build_lib(verbose)
    build_hostcheck(verbose)
    return lib


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(sys.argv[sys.argv.index("--sanitize") + 1], verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
