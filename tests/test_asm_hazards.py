"""The grouped multiply-adds of the carry-free 28-bit core (fe28.hpp) are
inline-asm blocks whose first v_mad_u64_u32 writes a scratch carry-out SGPR
pair before the later ones read their factors; a factor held in an SGPR (a
limb of p) must therefore never share a register with that pair.  The
constraint says so ("=&s"); this test checks the compiler's gfx950 assembly
of every translation unit that uses the core, so that a change to the
constraints, or a compiler that ignores them, fails here on the CPU rather
than as wrong sums on the GPU.  (Before the constraint was early-clobber, one
build of the merge kernel placed a carry-out on a limb of p and the buckets
it merged came out wrong.)"""

import concurrent.futures as cf
import os
import re
import shutil
import subprocess

import pytest

from paper_2502_11660_amd import build as B

UNITS = ["k_accum.hip", "k_agg.hip", "k_chain.hip", "k_elementwise.hip"]
MAD = re.compile(r"v_mad_u64_u32 v\[\d+:\d+\], s\[(\d+):(\d+)\], (\S+?),? (\S+?),")


def hazards(asm_text):
    """(block line, instruction) pairs where a v_mad_u64_u32 of an inline-asm
    block reads an SGPR that an earlier multiply-add of the same block wrote
    as its carry-out."""
    lines = asm_text.split("\n")
    found = []
    i = 0
    while i < len(lines):
        if "ASMSTART" in lines[i]:
            j = i + 1
            written = set()
            while "ASMEND" not in lines[j]:
                m = MAD.match(lines[j].strip())
                if m:
                    for op in (m.group(3), m.group(4)):
                        r = re.match(r"s(\d+)$", op)
                        if r and int(r.group(1)) in written:
                            found.append((j + 1, lines[j].strip()))
                    written |= {int(m.group(1)), int(m.group(2))}
                j += 1
            i = j
        i += 1
    return found


def test_scanner_catches_a_planted_overlap():
    """A hand-written block with the overlap, and the same block without."""
    bad = "\n".join([
        ";;#ASMSTART",
        "v_mad_u64_u32 v[70:71], s[10:11], v107, s7, v[70:71]",
        "v_mad_u64_u32 v[70:71], s[10:11], v111, s11, v[70:71]",
        ";;#ASMEND"])
    good = bad.replace("s11, v[70:71]", "s12, v[70:71]")
    assert len(hazards(bad)) == 1
    assert hazards(good) == []


@pytest.mark.skipif(shutil.which(B.hipcc()) is None and not os.path.exists(B.hipcc()),
                    reason="hipcc not available")
def test_no_carry_out_overlaps_an_sgpr_factor(tmp_path):
    cc = B.hipcc()
    inc = ["-I", os.path.join(B.ROOT, "include"), "-I", B.CSRC]

    def asm_of(unit):
        out = tmp_path / (unit + ".s")
        subprocess.run([cc, *B.HIPCC_FLAGS, *inc, "--cuda-device-only", "-S", "-o", str(out),
                        os.path.join(B.CSRC, unit)], check=True, capture_output=True)
        return unit, out.read_text()

    with cf.ThreadPoolExecutor(len(UNITS)) as ex:
        results = list(ex.map(asm_of, UNITS))
    for unit, text in results:
        assert "ASMSTART" in text, unit  # the core's asm blocks are there
        assert hazards(text) == [], unit
