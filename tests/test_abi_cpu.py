"""Host-side checks of the C ABI that need no GPU: the shared library loads and
exports every entry point the public header declares, and the Python binding
names the same set."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtlbl.h")
LIB = os.path.join(ROOT, "paper_cs_0703028_amd", "librtlbl.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("rt_setup_grid", "rt_setup_lines", "rt_compute_kappa", "rt_trace_rays", "rt_tally"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="librtlbl.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def declared_types():
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return set(re.findall(r"\}\s*(rt_[a-z_]+)\s*;", src)) | {"rt_ctx"}


def test_binding_uses_only_declared_symbols():
    src = open(os.path.join(ROOT, "paper_cs_0703028_amd", "rtlbl.py")).read()
    used = set(re.findall(r"\b(rt_[a-z_]+)\b", src))
    allowed = set(declared()) | declared_types()
    assert used <= allowed, used - allowed


def test_product_does_not_reach_the_oracle():
    pkg = os.path.join(ROOT, "paper_cs_0703028_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle|rt_oracle|orc_", text, re.M), f


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU; asking for more exits with a message."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
