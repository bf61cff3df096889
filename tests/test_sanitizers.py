"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

- The FP64 oracle (oracle/mjp_oracle.c) compiled with gcc's sanitizers and
  driven over every model, the degenerate cases and invalid arguments
  (tests/sanitize/oracle_driver.c).
- The library's host code (argument validation, operator checks, the host
  model generator and counter-based generator, error reporting) compiled
  with the sanitizers on the host side only -- its device code is compiled
  without optimisation and never runs -- and driven by
  tests/sanitize/abi_driver.c through the C ABI on a machine without a GPU.

Both programs exit 0 only when every check holds; any sanitizer report
aborts them (recovery disabled), so a non-zero status is the failure."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", os.path.join(HERE, "oracle_driver.c"), "-lm", "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert "all checks passed" in r.stdout


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not available")
def test_library_host_code_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2312_05647_amd", "csrc")
    srcs = sorted(f for f in os.listdir(csrc) if f.endswith(".hip"))
    flags = ["--offload-arch=gfx950", "-g", "-std=c++17", "-fPIC",
             "-Xarch_host", "-O1", "-Xarch_device", "-O0",
             "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", csrc]
    objs = [str(tmp_path / (s[:-4] + ".o")) for s in srcs]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        list(ex.map(lambda so: _run([HIPCC, *flags, "-c", os.path.join(csrc, so[0]), "-o", so[1]], timeout=900),
                    zip(srcs, objs)))
    lib = str(tmp_path / "libmjp_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address,undefined",
          *objs, "-o", lib], timeout=300)
    exe = str(tmp_path / "abi_driver")
    _run([CLANG, "-g", "-O1", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "abi_driver.c"),
          "-L", str(tmp_path), "-lmjp_san", f"-Wl,-rpath,{tmp_path}", "-lm", "-o", exe], timeout=300)
    r = _run([exe], env=ENV, timeout=300)
    assert "all checks passed" in r.stdout
