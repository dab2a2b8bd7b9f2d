import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle._load()
    return oracle


_ISA_SOURCES = ("bz_kernels.hip", "bz_batch.hip", "bz_sched.hip")


@pytest.fixture(scope="session")
def isa_asm(tmp_path_factory):
    """gfx950 assembly of the HIP sources, compiled once per session (in parallel) for the
    compiled-code checks: {source name: assembly text}."""
    import shutil
    import subprocess
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc) and not shutil.which("hipcc"):
        pytest.skip("hipcc not installed")
    csrc = os.path.join(ROOT, "paper_1911_08963_amd", "csrc")
    out = tmp_path_factory.mktemp("isa")
    flags = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "--cuda-device-only", "-S", "-I", os.path.join(ROOT, "include")]

    def one(src):
        dst = out / (src + ".s")
        subprocess.run([hipcc, *flags, os.path.join(csrc, src), "-o", str(dst)], check=True, capture_output=True)
        return src, dst.read_text()

    with ThreadPoolExecutor(len(_ISA_SOURCES)) as ex:
        return dict(ex.map(one, _ISA_SOURCES))
