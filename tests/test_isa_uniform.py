"""The enumeration kernels broadcast values only from loops that all lanes run together (compiled code, CPU).

bz_enum_kernel (and the task bookkeeping kernels beside it) hand a value to the
whole wave with readfirstlane: the tile index, the polled task key, the cancel
word, the wave minimum. That is only sound where every lane of the wave runs
the same iterations. If a loop that contains a readfirstlane were left by the
lanes one at a time (a lane-dependent exit, compiled as a loop whose back edge
tests exec), lanes still inside would read a value from a lane that is no
longer in step: an earlier version of the kernel hung that way, with lanes
1-63 re-entering the tile body with tile 0 after the compiler threaded a
lane-0 branch through the loop.

This compiles the kernels to gfx950 assembly with hipcc, rebuilds each loop
from the compiler's loop annotations, and checks that no loop containing a
v_readfirstlane is closed by the back edge of a loop that lanes leave one at a
time: an s_cbranch_execnz to its header (the latch has removed the lanes that
left). (An s_cbranch_execz to the header is the compiler's "no lane active,
fall through" shortcut after branch relaxation, not a back edge lanes take
separately.) A small kernel with exactly the hazardous shape, compiled the same
way, checks that the analysis finds it.
"""
from __future__ import annotations

import collections
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1911_08963_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "--cuda-device-only", "-S"]

needs_hipcc = pytest.mark.skipif(not os.path.exists(HIPCC) and not shutil.which("hipcc"),
                                 reason="hipcc not installed")

# a loop whose exit depends on the lane, with a readfirstlane inside
PROBE = r"""
#include <hip/hip_runtime.h>
__global__ void probe_divergent_loop(unsigned *p, unsigned n) {
    unsigned i = threadIdx.x;
    while (i < n) {
        unsigned u = __builtin_amdgcn_readfirstlane(p[i]);
        p[i] += u;
        i += threadIdx.x + 1;
    }
}
"""


def _compile(src_path, out_path):
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), src_path, "-o", str(out_path)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out_path.read_text()


def divergent_loops_with_broadcast(asm: str, kernel_pattern: str):
    """(kernel, loop header) of every loop that holds a v_readfirstlane and is
    closed by an s_cbranch_execnz back to its header."""
    found = []
    kernels = re.findall(kernel_pattern, asm, re.M)
    for k in kernels:
        start = asm.index(k + ":")
        end = asm.index(".Lfunc_end", start)
        lines = asm[start:end].splitlines()
        blocks = []            # [label, first line, last line, innermost loop header]
        parent = {}            # loop header -> enclosing loop header
        cur = None
        for i, line in enumerate(lines):
            m = re.match(r"^(\.LBB\w+):", line)
            if m:
                if cur:
                    blocks.append(cur)
                hdr = None
                mm = re.search(r"Header=BB(\w+) Depth", line)
                if mm:
                    hdr = ".LBB" + mm.group(1)
                if "Loop Header" in line:
                    hdr = m.group(1)
                cur = [m.group(1), i, i, hdr]
                continue
            if cur is None:
                continue
            cur[2] = i
            if "Loop Header" in line:
                cur[3] = cur[0]
            mm = re.search(r"Parent Loop BB(\w+) Depth", line)
            if mm and cur[3] == cur[0]:
                parent.setdefault(cur[0], ".LBB" + mm.group(1))
        if cur:
            blocks.append(cur)
        members = collections.defaultdict(list)
        for b in blocks:
            h = b[3]
            while h:
                members[h].append(b)
                h = parent.get(h)
        for h, bl in members.items():
            body = [lines[j] for b in bl for j in range(b[1], b[2] + 1)]
            if not any("v_readfirstlane" in x and not x.strip().startswith(";") for x in body):
                continue
            back = re.compile(r"\s*s_cbranch_execnz\s+" + re.escape(h) + r"\b")
            if any(back.match(x) for x in body):
                found.append((k, h))
    return kernels, found


@needs_hipcc
def test_analysis_finds_a_divergent_loop(tmp_path):
    src = tmp_path / "probe.hip"
    src.write_text(PROBE)
    asm = _compile(str(src), tmp_path / "probe.s")
    kernels, found = divergent_loops_with_broadcast(asm, r"^(_Z\w*probe_divergent_loop\w*):")
    assert len(kernels) == 1
    assert found, "the probe's lane-dependent loop around a readfirstlane was not found"


def test_enumeration_kernels_broadcast_in_uniform_loops(isa_asm):
    asm = isa_asm["bz_kernels.hip"]
    kernels, found = divergent_loops_with_broadcast(asm, r"^(_ZN2bz\d+bz_\w+_kernel\w*):")
    assert sum("bz_enum_kernel" in k for k in kernels) >= 64
    # the launches of small-level tasks spanning level ends: W 1..8 x 2, 4, 8 slots
    # (16 up to W = 4) x statistics or not
    assert sum("bz_enum_levels_kernel" in k for k in kernels) == 56
    assert not found, found[:4]


def test_schedule_kernels_broadcast_in_uniform_loops(isa_asm):
    asm = isa_asm["bz_sched.hip"]
    kernels, found = divergent_loops_with_broadcast(asm, r"^(_ZN2bz\d+bz_sched_kernel\w*):")
    assert len(kernels) == 32
    assert not found, found[:4]


def test_batch_and_one_launch_kernels_broadcast_in_uniform_loops(isa_asm):
    """The batched kernel and the one-launch single-code kernel: their loops read the claim
    results and the task fields through readfirstlane and must be left by the whole wave."""
    asm = isa_asm["bz_batch.hip"]
    for pattern, count in ((r"^(_ZN2bz\d+bz_batch_kernel\w*):", 4), (r"^(_ZN2bz\d+bz_one_kernel\w*):", 4)):
        kernels, found = divergent_loops_with_broadcast(asm, pattern)
        assert len(kernels) == count
        assert not found, found[:4]
