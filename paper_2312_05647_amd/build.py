"""Build libmjp.so (HIP for gfx950) in the package directory.

    python -m paper_2312_05647_amd.build

Every source under csrc/ is compiled with hipcc for gfx950 only and linked
into one shared library with a C ABI (include/mjp.h).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

try:
    from . import asmcheck
except ImportError:  # run as a script
    import asmcheck

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmjp.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=off: the Kahan updates and the exact FP32 row sums of B
# depend on every product being rounded where the source rounds it; fused
# multiply-adds are written explicitly with fmaf.
# packed-fp32-ops disabled: no v_pk_*_f32 in any kernel.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-function"]


def _compile(src: str) -> str:
    """Compiles one source, keeping the device assembly the object is
    assembled from, and refuses kernels with a loop that holds a barrier
    and exits lane by lane (asmcheck)."""
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    base = os.path.splitext(os.path.basename(src))[0]
    cmd = [HIPCC, *FLAGS, "-save-temps=obj", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    temps = [os.path.join(OBJ, f) for f in os.listdir(OBJ)
             if f.startswith(base + "-hip-") or f.startswith(base + "-host-") or f.startswith(base + ".hip-hip-")]
    try:
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
        asm = os.path.join(OBJ, f"{base}-hip-amdgcn-amd-amdhsa-gfx950.s")
        bad = asmcheck.check_file(asm)
        if bad:
            raise RuntimeError(f"{src}: loops holding a barrier that exit lane by lane: {bad}")
    finally:
        for f in temps:
            os.remove(f)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
