"""The built library's matrix-core accumulation chains use one product shape each.

A 16x16x16 BF16 product that takes a 16x16x32 product's result as its accumulator input (or
the reverse) came out of the compiler with too few wait states between the two and returned
wrong sums on the GPU, so the kernels pair K chunks only in chains that are 32-deep throughout
(an odd chunk count gets a zero partner).  This test disassembles the gfx950 code objects of the
library built here and checks every accumulator read against the last write to those registers
in program order within each kernel (any other instruction writing them ends the chain).  No GPU
is needed."""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "..", "paper_2211_12709_amd", "libfno_mi355x.so")
OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"

MFMA = re.compile(r"v_mfma_f32_16x16x(16|32)_?bf16\S*\s+(\S+),\s*(\S+),\s*(\S+),\s*(\S+)")
WRITE = re.compile(r"(v_\w+|\w*_load\w*|ds_read\w*)\s+([va]\[\d+:\d+\]|[va]\d+)")
FUNC = re.compile(r"^[0-9a-f]+ <(.+)>:$")


def _regs(tok):
    m = re.match(r"([va])\[(\d+):(\d+)\]$", tok)
    if m:
        return [f"{m.group(1)}{i}" for i in range(int(m.group(2)), int(m.group(3)) + 1)]
    return [tok] if re.match(r"[va]\d+$", tok) else []


def mixed_chains(lines):
    """(kernel, instruction) of every BF16 product whose accumulator was last written by a
    product of the other depth; also the number of 32-deep products seen."""
    last, bad, n32, func = {}, [], 0, None
    for raw in lines:
        line = raw.split("//")[0].strip()
        m = FUNC.match(raw.strip())
        if m:
            func, last = m.group(1), {}
            continue
        m = MFMA.match(line)
        if m:
            kind, dst, srcc = m.group(1), m.group(2), m.group(5)
            n32 += kind == "32"
            if any(last.get(r) not in (None, kind) for r in _regs(srcc)):
                bad.append((func, line))
            for r in _regs(dst):
                last[r] = kind
            continue
        m = WRITE.match(line)
        if m and not m.group(1).startswith(("v_cmp", "v_mfma")):
            for r in _regs(m.group(2)):
                last[r] = None
    return bad, n32


def test_scanner_catches_a_planted_mix():
    lines = ["0000000000001000 <k>:",
             "\tv_mfma_f32_16x16x32_bf16 a[0:3], v[4:7], v[8:11], a[0:3]// 0: 0",
             "\tv_mfma_f32_16x16x16_bf16 a[0:3], v[4:5], v[8:9], a[0:3]  // 0: 0"]
    assert len(mixed_chains(lines)[0]) == 1
    # a move into the accumulator registers in between starts a new chain
    fixed = lines[:2] + ["\tv_accvgpr_write_b32 a0, 0", "\tv_accvgpr_write_b32 a1, 0",
                         "\tv_accvgpr_write_b32 a2, 0", "\tv_accvgpr_write_b32 a3, 0"] + lines[2:]
    assert mixed_chains(fixed)[0] == []


@pytest.mark.skipif(not (os.path.exists(LIB) and os.path.exists(OBJDUMP)),
                    reason="library not built here, or no llvm-objdump")
def test_no_mixed_depth_chains_in_the_built_library(tmp_path):
    lib = tmp_path / "lib.so"
    shutil.copy(LIB, lib)
    subprocess.run([OBJDUMP, "--offloading", str(lib)], check=True, capture_output=True, cwd=tmp_path)
    objs = sorted(p for p in tmp_path.iterdir() if p.name.endswith("gfx950"))
    assert objs, "no gfx950 code object in the library"
    bad, n32 = [], 0
    for obj in objs:
        out = subprocess.run([OBJDUMP, "-d", "--mcpu=gfx950", str(obj)], check=True, capture_output=True,
                             text=True).stdout
        b, n = mixed_chains(out.splitlines())
        bad += b
        n32 += n
    assert n32 > 0, "no 16x16x32 products found: the disassembly format is not the one parsed"
    assert bad == [], bad[:5]
