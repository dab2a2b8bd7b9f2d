"""The persistent and schedule kernels issue each atomic from one lane (compiled code check, CPU).

Work claims, completions and log appends are wave-wide operations on a few hot
words. Each must reach memory as one atomic per wave: an atomic executed by
all 64 lanes multiplies the traffic on those cache lines by 64 (the search
stays correct but runs several times slower). This compiles the batch/serving
kernels to gfx950 assembly with hipcc and checks every global atomic of the
persistent kernels: it must sit in a single-lane region, either a lane-0
branch (mbcnt election or saveexec, or a lane-0 mask hoisted out of a loop) or
the explicit exec narrowing of the wave-atomic helpers. (The GPU tests, which
compare combination counts exactly, catch an atomic that runs on every lane.)
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1911_08963_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.parametrize("source,pattern,count", [
    ("bz_batch.hip", r"^(_ZN2bz\d+bz_(?:batch|serve)_kernel\w+):", 6),
    ("bz_sched.hip", r"^(_ZN2bz\d+bz_sched_kernel\w+):", 32),
])
def test_persistent_kernel_atomics_are_single_lane(isa_asm, source, pattern, count):
    s = isa_asm[source]
    kernels = re.findall(pattern, s, re.M)
    assert len(kernels) == count
    for k in kernels:
        body = s[s.index(k + ":"):s.index(".Lfunc_end", s.index(k + ":"))].splitlines()
        n = 0
        for i, line in enumerate(body):
            if "_atomic_" not in line or line.strip().startswith(";"):
                continue
            n += 1
            ctx = " ".join(body[max(0, i - 24):i])
            # lane-0 regions: an mbcnt election or saveexec, the helpers' exec
            # narrowing, or a lane-0 mask the compiler hoisted out of the loop and
            # reapplies with s_and_b64 + s_mov_b64 exec
            hoisted = "s_and_b64" in ctx and "s_mov_b64 exec, s[" in ctx
            assert ("v_mbcnt" in ctx or "s_and_saveexec" in ctx or "s_lshl_b64 exec" in ctx or hoisted), \
                f"{k}: atomic without a single-lane region: {line.strip()}"
        assert n > 0
