"""Device code of the built library: no FP64 instruction anywhere.

The precision contract keeps FP64 off the GPU: host code forms the FP64
quantities (the Eq. 8 basis, camera frames) and hands FP32 to the kernels.
This test reads the gfx950 code objects that the build embedded in libfpo.so
(the .hip_fatbin section holds one offload bundle per HIP source),
disassembles them with the ROCm LLVM tools and checks that no VALU
instruction takes or produces an f64 operand.  Library calls are included,
which is what catches a math routine that widens internally.
"""
from __future__ import annotations

import os
import re
import struct
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2202_08614_amd", "libfpo.so")
LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def _code_objects(tmp_path):
    fat = tmp_path / "fatbin.bin"
    subprocess.check_call([f"{LLVM}/llvm-objcopy", "--dump-section", f".hip_fatbin={fat}", LIB,
                           str(tmp_path / "stripped.so")])
    blob = fat.read_bytes()
    out = []
    i = blob.find(MAGIC)
    while i >= 0:
        (n_entries,) = struct.unpack_from("<Q", blob, i + len(MAGIC))
        p = i + len(MAGIC) + 8
        for _ in range(n_entries):
            off, size, tlen = struct.unpack_from("<QQQ", blob, p)
            p += 24
            triple = blob[p:p + tlen].decode()
            p += tlen
            if "gfx950" in triple and size > 0:
                out.append(blob[i + off:i + off + size])
        i = blob.find(MAGIC, i + len(MAGIC))
    return out


@pytest.mark.skipif(not (os.path.exists(LIB) and os.path.exists(f"{LLVM}/llvm-objdump")),
                    reason="needs the built library and the ROCm LLVM tools")
def test_no_fp64_instruction_in_device_code(tmp_path):
    objs = _code_objects(tmp_path)
    assert len(objs) >= 6, "expected one gfx950 code object per HIP source"
    f64 = re.compile(r"^\s+v_\w*f64\w*", re.M)
    found = []
    n_insts = 0
    for k, co in enumerate(objs):
        path = tmp_path / f"co{k}.elf"
        path.write_bytes(co)
        asm = subprocess.run([f"{LLVM}/llvm-objdump", "-d", "--mcpu=gfx950", str(path)], check=True,
                             capture_output=True, text=True).stdout
        n_insts += len(re.findall(r"^\s+[sv]_\w+", asm, re.M))
        found += f64.findall(asm)
    assert n_insts > 10000, "disassembly looks empty"
    assert not found, f"FP64 instructions in device code: {sorted(set(s.strip() for s in found))}"
