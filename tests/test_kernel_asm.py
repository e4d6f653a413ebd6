"""Properties of the compiled binary32 pair kernel (gfx950 assembly, built on the CPU).

The vector register file of a gfx950 SIMD has four banks (register number
mod 4). A v_fma_f32 whose two multiplicands sit in one bank issues in about
4.4 cycles per wave64 instruction, one with its three sources in three
banks in about 2.8 (the issue-rate probe, kinds 21 and 22). The filter's
multiply-adds take an entry component and a query component; the query is
staged as (T, -2C) so that component k of the two vectors lands in
different banks. This test keeps that property from silently regressing
when the kernel or the compiler changes the register assignment.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_1405_7461_amd import build as B

HIPCC = B.HIPCC


def _asm(tmp_path):
    out = tmp_path / "tds_kernels.s"
    cmd = [HIPCC, *B.COMMON, "--cuda-device-only", "-S", str(B.CSRC / "tds_kernels.hip"), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


def _kernel_body(text, prefix):
    m = re.search(r"^(" + re.escape(prefix) + r"\w*):", text, re.M)
    assert m, prefix
    end = text.index(".Lfunc_end", m.end())
    return m.group(1), text[m.end():end]


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which(HIPCC)), reason="hipcc not available")
def test_filter_multiply_adds_read_two_banks(tmp_path):
    text = _asm(tmp_path)
    # k_pair<kModeFP32Refine, 256 threads, EPT entries per lane, no overlap count>
    name, body = _kernel_body(text, "_ZN3tds6k_pairILi1ELi256ELi")
    ops = re.findall(r"v_(?:fma|fmac)_f32(?:_e32|_e64)?\s+v\d+,\s*v(\d+),\s*v(\d+)", body)
    assert len(ops) >= 24, (name, len(ops))  # the filter's multiply-adds are there
    same = [(a, b) for a, b in ops if int(a) % 4 == int(b) % 4]
    assert not same, f"{name}: {len(same)} of {len(ops)} multiply-adds read both multiplicands from one bank"
