"""Build libbz.so (HIP kernels for gfx950 plus the host library) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libbz.so")
SOURCES = ["bz_api.cpp", "bz_prepare.cpp", "bz_plan.cpp", "bz_kernels.hip", "bz_batch.hip",
           "bz_server.cpp", "bz_tune.cpp",
           "bz_count.hip", "bz_count.cpp", "bz_sched.hip", "bz_sched.cpp", "bz_noalloc.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-pthread",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = ("packed-fp32-ops", "hip-link")
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if l.strip() and not any(x in l for x in noise)]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))


def build(verbose: bool = False) -> str:
    """Compiles every source to an object in parallel (a few at a time), then links libbz.so."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    compile_flags = [f for f in FLAGS if f != "-shared"]
    inc = ["-I", os.path.join(ROOT, "include")]
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", "0") or 0) or (os.cpu_count() or 1), 16))
    with tempfile.TemporaryDirectory(prefix="bz_build_") as tmpdir:
        objs = [os.path.join(tmpdir, s + ".o") for s in SOURCES]          # bz_x.hip and bz_x.cpp both exist
        cmds = [[HIPCC, *compile_flags, *inc, "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        tmp = LIB + ".tmp"
        _run([HIPCC, *FLAGS, "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
