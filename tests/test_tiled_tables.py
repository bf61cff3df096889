"""Host logic of the tiled sweep (CPU only): the tables `build_mj_table`
makes for stencil plans of the two-species cascade, checked and emulated
by tests/host/tiled_tables.cpp, which includes the library source (its
device code is compiled without optimisation and never runs).  Shapes:
square, oblong and ragged-size grids, thin grids, a band operator (one
grid row), and both jump counts per synchronisation."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC) or shutil.which("g++") is None,
                                reason="ROCm compiler not available")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("tiled") / "tiled_tables")
    csrc = os.path.join(ROOT, "paper_2312_05647_amd", "csrc")
    cmd = [HIPCC, "--offload-arch=gfx950", "-std=c++17", "-Xarch_host", "-O2", "-Xarch_device", "-O0",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(ROOT, "tests", "host", "tiled_tables.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout + r.stderr
    return exe


@pytest.mark.parametrize("shape", [(1000, 1000, 256, 8), (1000, 1000, 256, 4), (997, 1003, 256, 8),
                                   (700, 1100, 256, 8), (130, 77, 256, 8), (4096, 1, 256, 8),
                                   (200000, 1, 256, 8), (2000, 500, 256, 4)])
def test_tiled_tables(driver, shape):
    r = subprocess.run([driver, *map(str, shape), "2"], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "stale reads=0 max |tiled - whole| = 0" in r.stdout
