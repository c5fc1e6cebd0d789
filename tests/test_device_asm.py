"""Properties of the gfx950 device code, read from the assembly hipcc emits
for the library's kernel sources with the library's own flags (no GPU
needed):

* no packed fp32 add, multiply or fma anywhere (every source is built with
  packed-fp32 selection off; hand-written forms are not used either);
* no scratch memory in any kernel (no register spills, no private arrays);
* the resident kernel's coherent accesses carry the cache hints it was
  measured best with: pixel rows and coefficient runs are read with agent-
  scope coherent loads and no streaming hint, and its outputs are written
  through L2 with the streaming hint;
* the batch and plain kernels stream every 16-byte coefficient access with
  the non-temporal hint.
"""
import importlib.util
import os
import re
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from conftest import ROOT

SOURCES = ["tdct_kernels.hip", "tdct_resident.hip", "tdct_probe.hip"]


def _build_module():
    spec = importlib.util.spec_from_file_location(
        "tdct_build", os.path.join(ROOT, "paper_1702_00817_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    b = _build_module()
    if not shutil.which(b.HIPCC) and not os.path.exists(b.HIPCC):
        pytest.skip("hipcc not found")
    out = tmp_path_factory.mktemp("asm")

    def compile_one(name):
        dst = os.path.join(str(out), name + ".s")
        cmd = ([b.HIPCC] + b.COMMON + ["-x", "hip"] + b.DEVICE + b.PER_SOURCE.get(name, [])
               + ["--offload-device-only", "-S", "-o", dst, os.path.join(b.CSRC, name)])
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        assert r.returncode == 0, r.stdout[-2000:]
        with open(dst) as f:
            return name, f.read()

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        return dict(ex.map(compile_one, SOURCES))


def _instructions(text, mnemonic):
    """The operand text of every `mnemonic` instruction (comments cut)."""
    pat = re.compile(r"^\s*" + re.escape(mnemonic) + r"\s+([^;\n]*)", re.M)
    return [m.group(1).strip() for m in pat.finditer(text)]


def test_no_packed_fp32_arithmetic(asm):
    for name, text in asm.items():
        for op in ("v_pk_add_f32", "v_pk_mul_f32", "v_pk_fma_f32"):
            assert op not in text, (name, op)


def test_no_scratch_in_any_kernel(asm):
    for name, text in asm.items():
        sizes = re.findall(r";\s*ScratchSize:\s*(\d+)", text)
        assert sizes, name
        assert all(s == "0" for s in sizes), (name, sizes)


def test_resident_kernel_cache_hints(asm):
    text = asm["tdct_resident.hip"]
    # pixel rows: 8-byte accesses through a 64-bit per-lane address
    row_loads = [o for o in _instructions(text, "global_load_dwordx2") if ", off" in o]
    row_stores = [o for o in _instructions(text, "global_store_dwordx2") if ", off" in o]
    assert row_loads and row_stores
    assert all("sc1" in o.split() and "nt" not in o.split() for o in row_loads), row_loads
    assert all({"sc1", "nt"} <= set(o.split()) for o in row_stores), row_stores
    # coefficient runs and job copies: 16-byte buffer accesses
    loads = _instructions(text, "buffer_load_dwordx4")
    stores = _instructions(text, "buffer_store_dwordx4")
    assert loads and stores
    assert all("sc1" in o.split() and "nt" not in o.split() for o in loads), loads
    assert all({"sc1", "nt"} <= set(o.split()) for o in stores), stores
    # byte-wise rows (unaligned planes) are coherent too
    for op in ("global_load_ubyte", "global_store_byte"):
        rows = [o for o in _instructions(text, op) if ", off" in o]
        assert all("sc1" in o.split() for o in rows), (op, rows)


def test_batch_and_plain_kernels_stream_coefficients(asm):
    text = asm["tdct_kernels.hip"]
    loads = _instructions(text, "global_load_dwordx4")
    stores = _instructions(text, "global_store_dwordx4")
    assert loads and stores
    assert all("nt" in o.split() for o in loads), [o for o in loads if "nt" not in o.split()][:4]
    assert all("nt" in o.split() for o in stores), [o for o in stores if "nt" not in o.split()][:4]
