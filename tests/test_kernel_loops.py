"""Static check of the gfx950 code: no lane exchange inside a divergent loop.

Wavefront-cooperative kernels broadcast values between lanes (ds_bpermute,
DPP, swizzle).  If the compiler builds a loop around such an exchange with a
per-lane exit (the loop's exit mask is updated with ``s_andn2_b64 exec,
exec, ...``), lanes can leave the loop at different iterations and the
remaining lanes then read registers of lanes that are masked off -- a
broadcast of the item index from an inactive lane 0 spins forever.  Every
loop that holds a lane exchange must therefore branch as a whole (scalar
condition), which this test checks on the device assembly of each source
compiled with the library's own flags.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess

import pytest

from paper_2409_08975_amd import build as B

HIPCC = B.HIPCC
EXCHANGE = re.compile(r"ds_bpermute|ds_swizzle|row_shr|row_shl|row_ror|row_bcast|row_mirror|"
                      r"row_half_mirror|quad_perm|v_permlane|wave_shr|wave_ror")
DIVERGENT_EXIT = re.compile(r"s_andn2_b64 exec, exec")


def parse_loops(asm: str):
    """{kernel: [(header, own_lines, all_lines)]} from LLVM's loop annotations."""
    out = {}
    kernel = None
    blocks, order, header_of, parent_of = {}, [], {}, {}

    def finish():
        if kernel is None:
            return
        loops = {}
        for b in order:
            h, seen = header_of.get(b), set()
            while h is not None and h not in seen:
                seen.add(h)
                loops.setdefault(h, []).append(b)
                h = parent_of.get(h)
        out[kernel] = [(h, [ln for b in mem if header_of.get(b) == h for ln in blocks[b]],
                        [ln for b in mem for ln in blocks[b]]) for h, mem in loops.items()]

    for line in asm.split("\n"):
        m = re.match(r"^(_Z\w+):", line)
        if m:
            finish()
            kernel = m.group(1)
            blocks, order, header_of, parent_of = {"entry": []}, ["entry"], {}, {}
            cur = "entry"
            continue
        if kernel is None:
            continue
        m = re.match(r"^(\.LBB\d+_\d+|; %bb\.\d+):\s*(;.*)?$", line)
        if m:
            cur = m.group(1)
            blocks[cur] = []
            order.append(cur)
            note = m.group(2) or ""
            mh = re.search(r"Header=BB(\d+_\d+)", note)
            if mh:
                header_of[cur] = ".LBB" + mh.group(1)
            if "Loop Header" in note:
                header_of[cur] = cur
            mp = re.search(r"Parent Loop BB(\d+_\d+)", note)
            if mp:
                parent_of[cur] = ".LBB" + mp.group(1)
            continue
        blocks[cur].append(line)
    finish()
    return out


def divergent_exchange_loops(asm: str):
    bad = []
    for kernel, loops in parse_loops(asm).items():
        for header, own, body in loops:
            if any(DIVERGENT_EXIT.search(ln) for ln in own) and \
                    any(EXCHANGE.search(ln) for ln in body):
                bad.append((kernel, header))
    return bad


SAMPLE_BAD = """
_ZN2tc4kbadEv:
\ts_mov_b64 s[4:5], 0
.LBB0_1:                                ; =>This Inner Loop Header: Depth=1
\tds_bpermute_b32 v2, v1, v2
\ts_andn2_b64 exec, exec, s[4:5]
\ts_cbranch_execnz .LBB0_1
\ts_endpgm
_ZN2tc5kgoodEv:
.LBB1_1:                                ; =>This Inner Loop Header: Depth=1
\tds_bpermute_b32 v2, v1, v2
\ts_cmp_ge_u32 s2, s3
\ts_cbranch_scc0 .LBB1_1
.LBB1_2:                                ; =>This Inner Loop Header: Depth=1
\tv_add_u32 v3, 1, v3
\ts_andn2_b64 exec, exec, s[6:7]
\ts_cbranch_execnz .LBB1_2
\ts_endpgm
"""


def test_parser_flags_divergent_exchange_only():
    assert divergent_exchange_loops(SAMPLE_BAD) == [("_ZN2tc4kbadEv", ".LBB0_1")]


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC),
                    reason="hipcc not available")
@pytest.mark.parametrize("source", B.SOURCES)
def test_no_lane_exchange_in_divergent_loop(source, tmp_path):
    flags = [f for f in B.FLAGS if f not in ("-shared", "-fPIC")]
    out = tmp_path / (source + ".s")
    subprocess.run([HIPCC] + flags + ["--cuda-device-only", "-S",
                                      os.path.join(B.CSRC, source), "-o", str(out)],
                   check=True, capture_output=True)
    asm = out.read_text()
    assert "Loop Header" in asm or "k_" not in asm
    assert divergent_exchange_loops(asm) == []
