"""The C ABI library loads and exports every entry point include/hrest.h
declares; the oracle and the product share no code.  CPU only (no compute
calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hrest.h")
LIB = os.path.join(ROOT, "paper_2412_03489_amd", "libhrest.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hr_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_estimator_calls():
    names = declared()
    for must in ("hr_est_grad", "hr_est_hessian", "hr_est_hvp", "hr_newton_cg_step"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhrest.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    import paper_2412_03489_amd as P
    assert set(P.EXPORTED) == set(declared())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhrest.so not built")
def test_library_is_gfx950_code_object():
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", LIB], capture_output=True, text=True)
    if out.returncode != 0:
        pytest.skip("roc-obj-ls unavailable")
    assert "gfx950" in out.stdout


def test_library_links_roctx_for_marker_ranges():
    """The host-side calls carry roctx ranges (rocprofv3 --marker-trace): the
    library links the roctx library and exports nothing of it."""
    import shutil
    import subprocess
    if shutil.which("readelf") is None:
        pytest.skip("readelf not installed")
    out = subprocess.run(["readelf", "-d", LIB], check=True, capture_output=True, text=True).stdout
    assert "librocprofiler-sdk-roctx" in out
    syms = subprocess.run(["readelf", "--dyn-syms", "-W", LIB], check=True, capture_output=True,
                          text=True).stdout
    assert "roctxRangePushA" in syms   # imported (undefined here), resolved at load time


def test_oracle_and_product_share_no_code():
    pkg = os.path.join(ROOT, "paper_2412_03489_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in txt and "orc.h" not in txt and "liborc" not in txt, fn
    otxt = open(os.path.join(ROOT, "oracle", "orc.c")).read() + open(
        os.path.join(ROOT, "oracle", "__init__.py")).read()
    for needle in ("hrest.h", "libhrest", "import paper_2412_03489_amd",
                   "from paper_2412_03489_amd", "hr_device.h", "hr_kernels.h"):
        assert needle not in otxt, needle


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import importlib

    import paper_2412_03489_amd as P
    monkeypatch.setattr(P, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(P, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        P.lib()
    importlib.reload(P)


# ctypes mirror of each public struct in the binding, by C type name
_STRUCTS = {"hr_opts": "Opts", "hr_ncg_opts": "NcgOpts", "hr_ncg_report": "NcgReport",
            "hr_optim_opts": "OptimOpts", "hr_query": "Query", "hr_batch_opts": "BatchOpts",
            "hr_batch_report": "BatchReport", "hr_server_opts": "ServerOpts",
            "hr_query_stats": "QueryStats", "hr_server_stats": "ServerStats"}


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    the C compiler gives the header's struct (gcc, no GPU)."""
    import ctypes
    import re
    import subprocess

    import paper_2412_03489_amd as P
    hdr = open(os.path.join(ROOT, "include", "hrest.h")).read()
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "hrest.h"', "int main(void) {"]
    for cname, pname in _STRUCTS.items():
        py = getattr(P, pname)
        assert re.search(r"\}\s*" + cname + r"\s*;", hdr), cname
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln.strip():
            c, f, v = ln.split()
            got[(c, f)] = int(v)
    for cname, pname in _STRUCTS.items():
        py = getattr(P, pname)
        assert ctypes.sizeof(py) == got[(cname, "size")], cname
        for fname, _ in py._fields_:
            assert getattr(py, fname).offset == got[(cname, fname)], (cname, fname)
