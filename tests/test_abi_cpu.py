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


def header_constants():
    """RT_* enumerators and #defines of the public header, with their values."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    vals = {n: int(v) for n, v in re.findall(r"\b(RT_[A-Z0-9_]+)\s*=\s*(-?\d+)", src)}
    vals.update({n: int(v) for n, v in re.findall(r"#define\s+(RT_[A-Z0-9_]+)\s+(-?\d+)\b", src)})
    return vals


def test_binding_constants_match_the_header():
    # the binding mirrors the header's constants, either under the same name
    # or without the RT_ prefix; every kappa mode is mirrored
    import ast
    tree = ast.parse(open(os.path.join(ROOT, "paper_cs_0703028_amd", "rtlbl.py")).read())
    py = {}
    for node in tree.body:
        if isinstance(node, ast.Assign):
            targets = node.targets[0]
            names = [t.id for t in (targets.elts if isinstance(targets, ast.Tuple) else [targets])
                     if isinstance(t, ast.Name)]
            try:
                value = ast.literal_eval(node.value)
            except ValueError:
                continue
            if names == ["ARITH_OPS"]:
                # rt_arith_op codes: op name -> (code, operands read)
                py.update({"RT_AR_" + k.upper(): v[0] for k, v in value.items()})
                continue
            values = value if isinstance(value, tuple) else (value,)
            if len(values) == len(names):
                py.update(zip(names, values))
    hdr = header_constants()
    modes = [n for n in hdr if n.startswith("RT_KAPPA_")]
    assert "RT_KAPPA_ADAPTIVE_WINGS" in modes
    checked = 0
    for name, v in hdr.items():
        for alias in (name, name[3:]):
            if alias in py:
                assert py[alias] == v, (name, alias, py[alias], v)
                checked += 1
    for m in modes:
        assert m[3:] in py or m in py, m
    ops = [n for n in hdr if n.startswith("RT_AR_")]
    assert ops and all(n in py for n in ops)
    assert checked == len(hdr), sorted(set(hdr) - {n for n in hdr if n in py or n[3:] in py})
