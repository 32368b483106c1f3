"""Checks of the device code itself (no GPU needed).

Two constructs are kept out of every kernel of libesc.so:

* inline assembly: the compiler cannot see hazards inside an asm block or
  between it and the code around it;
* 64-bit shifts (v_lshlrev_b64, v_lshrrev_b64, v_ashrrev_i64) whose shift
  amount is a VGPR.  A documented gfx90a erratum makes such a shift read a
  wrong amount when the amount sits in the highest allocated VGPR; the
  installed compiler works around it for gfx90a only, not for gfx950.  The
  split-selectivity kernel gave silent run-to-run count differences while
  its 64-bit bitset test shifted by a register amount held in the kernel's
  highest VGPR; the kernels now use 32-bit words, mbcnt and constant
  amounts.

The second check disassembles the gfx950 code objects embedded in the built
library (the fat-binary section), so it covers what actually ships.
"""
import os
import re
import struct
import subprocess

import pytest

from paper_1901_01488_amd import esc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1901_01488_amd", "csrc")
LLVM = "/opt/rocm/llvm/bin"
BUNDLE_MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
SHIFT64 = re.compile(r"\b(v_lshlrev_b64|v_lshrrev_b64|v_ashrrev_i64)\s+(\S+),\s*([^,\s]+),")


def device_sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".h", ".cpp")))


def test_no_inline_assembly_in_sources():
    pat = re.compile(r"\b(asm|__asm__|__asm)\b\s*(volatile|__volatile__)?\s*\(")
    hits = []
    for path in device_sources():
        code = re.sub(r"//[^\n]*|/\*.*?\*/", "", open(path).read(), flags=re.S)
        for m in pat.finditer(code):
            hits.append((os.path.basename(path), code[:m.start()].count("\n") + 1))
    assert not hits, hits


def gfx950_code_objects(lib_path, tmp_path):
    """The gfx950 code objects of the library's offload bundles, as files."""
    fat = tmp_path / "fatbin.bin"
    subprocess.run([os.path.join(LLVM, "llvm-objcopy"), "--dump-section", f".hip_fatbin={fat}", lib_path,
                    str(tmp_path / "lib.copy")], check=True, capture_output=True)
    data = fat.read_bytes()
    out = []
    start = data.find(BUNDLE_MAGIC)
    while start >= 0:
        nentries = struct.unpack_from("<Q", data, start + len(BUNDLE_MAGIC))[0]
        pos = start + len(BUNDLE_MAGIC) + 8
        for _ in range(nentries):
            off, size, tlen = struct.unpack_from("<QQQ", data, pos)
            triple = data[pos + 24:pos + 24 + tlen].decode()
            pos += 24 + tlen
            if triple.endswith("gfx950") and size:
                path = tmp_path / f"co{len(out)}.elf"
                path.write_bytes(data[start + off:start + off + size])
                out.append(path)
        start = data.find(BUNDLE_MAGIC, start + 1)
    return out


def test_no_register_amount_64bit_shifts_in_built_kernels(tmp_path):
    lib_path = esc.lib()._name
    objs = gfx950_code_objects(lib_path, tmp_path)
    assert len(objs) >= 4, "expected the scan, batch, join and MLP code objects"
    nshift = 0
    bad = []
    for co in objs:
        dis = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", "--mcpu=gfx950", str(co)],
                             check=True, capture_output=True, text=True).stdout
        assert "s_endpgm" in dis
        for line in dis.splitlines():
            m = SHIFT64.search(line)
            if not m:
                continue
            nshift += 1
            if re.fullmatch(r"v\d+", m.group(3)):
                bad.append(line.strip())
    assert nshift > 0, "no 64-bit shift recognised: disassembly format changed?"
    assert not bad, bad[:10]
