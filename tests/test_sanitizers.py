"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU code.

* The oracle (plain C, gcc) with tests/sanitize_oracle.c, which calls every
  oracle entry point on small disk, path-traced, analytic and edge scenes with
  every sampler, the solvers, the optimiser and the grey-box compositions.
* The HIP library's host code (hipcc, sanitizers on the host pass only; the
  device code is built as usual and never runs here) with
  tests/sanitize_host.c, which exercises what runs without a GPU: option
  defaults, context creation on a host with no usable device, and the argument
  checks of every entry point.

Both must finish without a sanitizer report and without a leak.
"""
import glob
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{cmd[0]} failed ({r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_oracle")
    run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "oracle"),
         os.path.join(ROOT, "oracle", "orc.c"), os.path.join(TESTS, "sanitize_oracle.c"),
         "-lm", "-lpthread", "-o", exe])
    r = run([exe], env=SAN_ENV, timeout=300)
    assert "sanitize driver ok" in r.stdout


def test_host_library_under_asan_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_2412_03489_amd import build as B
    clang = "/opt/rocm/llvm/bin/clang++"
    if not (os.path.exists(B.HIPCC) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not installed")
    # sanitizers on the host pass only; -O1 keeps the device pass short
    flags = [f for f in B.FLAGS if f != "-O3"] + [
        "-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
        "-Xarch_host", "-fno-sanitize-recover=all"]
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2412_03489_amd", "csrc", "*.hip")))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        run([B.HIPCC, *flags, "-c", src, "-o", obj])
        return obj

    with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    drv = str(tmp_path / "sanitize_host.o")
    run([clang.replace("clang++", "clang"), "-g", "-Wall", "-fsanitize=address,undefined",
         "-I", os.path.join(ROOT, "include"), "-c", os.path.join(TESTS, "sanitize_host.c"),
         "-o", drv])
    exe = str(tmp_path / "sanitize_host")
    run([clang, "-fsanitize=address,undefined", "-o", exe, drv, *objs, *B.LIBS, "-lamdhip64",
         "-lpthread"])
    r = run([exe], env=SAN_ENV, timeout=300)
    assert "sanitize host driver ok" in r.stdout
