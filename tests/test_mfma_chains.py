"""The device code keeps every MFMA accumulator chain in one instruction form.

The network runs on two bf16 MFMA forms, 16x16x16 and CDNA4's 16x16x32.  The
compiler issues an MFMA that takes as C the result of the previous MFMA
directly behind it, and where the two differ in form the sum misses part of
the first product: the backward product through W3 once ended its chain with
16x16x16 steps behind a 16x16x32, and its gradient came out wrong by up to
40 % (relative norm), by an amount that moved with the schedule.  The
kernels avoid the pattern by construction; this test reads the gfx950
assembly of the two translation units that hold MFMAs (built here with the
library's own flags) and checks that no MFMA takes as C a register last
written by an MFMA of the other form.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_1705_04702_amd import build as B

REG = re.compile(r"([av])\[(\d+):(\d+)\]|([av])(\d+)")


def _regs(tok):
    m = REG.fullmatch(tok.strip())
    if not m:
        return []
    if m.group(1):
        return [(m.group(1), r) for r in range(int(m.group(2)), int(m.group(3)) + 1)]
    return [(m.group(4), int(m.group(5)))]


def mixed_chains(asm: str):
    """(line, text) of every MFMA whose C operand was last written, in
    program order within one function, by an MFMA of another form.  Any
    other instruction that writes a register ends the chain on it (stores
    write memory, scalar instructions scalar registers)."""
    last, found = {}, []
    for i, line in enumerate(asm.splitlines()):
        if re.match(r"^_Z\w+:", line):
            last = {}
            continue
        m = re.match(r"\s+([a-z_0-9]+)\s+([^,\s]+)(.*)", line)
        if not m:
            continue
        op, dst, rest = m.groups()
        if op.startswith(("s_", ".")) or "store" in op or op.startswith("ds_write"):
            continue
        if op.startswith("v_mfma"):
            srcc = rest.split(",")[3]
            if any(last.get(r) not in (None, op) for r in _regs(srcc)):
                found.append((i + 1, line.strip()))
            for r in _regs(dst):
                last[r] = op
        else:
            for r in _regs(dst):
                last[r] = None
    return found


def test_scanner_flags_a_mixed_chain_and_passes_a_reloaded_one():
    mixed = """_ZN4mcrt1kEv:
	v_mfma_f32_16x16x32_bf16 a[112:115], v[6:9], v[16:19], 0
	v_add_u32_e32 v6, 0xa100, v128
	v_mfma_f32_16x16x16_bf16 a[112:115], v[160:161], v[2:3], a[112:115]
"""
    same = mixed.replace("16x16x16_bf16", "16x16x32_bf16").replace("v[160:161], v[2:3]", "v[160:163], v[2:5]")
    reloaded = """_ZN4mcrt1kEv:
	v_mfma_f32_16x16x16_bf16 v[20:23], v[22:23], v[2:3], v[158:161]
	ds_read_b128 v[20:23], v83 offset:256
	v_mfma_f32_16x16x32_bf16 v[20:23], v[158:161], v[12:15], v[20:23]
"""
    other_function = """_ZN4mcrt1aEv:
	v_mfma_f32_16x16x32_bf16 a[0:3], v[6:9], v[16:19], 0
_ZN4mcrt1bEv:
	v_mfma_f32_16x16x16_bf16 a[0:3], v[0:1], v[2:3], a[0:3]
"""
    assert [n for n, _ in mixed_chains(mixed)] == [4]
    assert mixed_chains(same) == []
    assert mixed_chains(reloaded) == []
    assert mixed_chains(other_function) == []


@pytest.mark.skipif(not os.path.exists(B.HIPCC) and not shutil.which("hipcc"), reason="hipcc not installed")
@pytest.mark.parametrize("unit", ["proposal.hip", "transport_f32.hip"])
def test_device_code_has_no_mixed_mfma_chains(unit, tmp_path):
    out = tmp_path / (unit + ".s")
    cmd = [B.HIPCC, *B.COMMON, "-x", "hip", "--cuda-device-only", "-S", os.path.join(B.CSRC, unit), "-o", str(out)]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout[-2000:]
    asm = out.read_text()
    assert asm.count("v_mfma_f32_16x16x32_bf16") > 0
    assert mixed_chains(asm) == []
