"""The Python binding's ctypes mirrors of the public structs of
include/rtlbl.h have the C compiler's layout: a C program built with gcc
against the header prints each struct's size and the offset of every field
the binding names, and they must equal the ctypes ones.  (A field added to
the header but not to the binding, or in another place, changes a size or an
offset; a field the header lacks fails to compile.)  Host only."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# ctypes class name in the binding -> C type name in the header
STRUCTS = {
    "RtStats": "rt_stats",
    "RtCase": "rt_case",
    "BatchTuning": "rt_batch_tuning",
    "SurrogateCfg": "rt_surrogate_cfg",
    "SurrogateStats": "rt_surrogate_stats",
}


def _binding_classes():
    """The ctypes classes, read from the binding's source without loading
    the GPU library (the module's import does)."""
    import ast
    src = open(os.path.join(ROOT, "paper_cs_0703028_amd", "rtlbl.py")).read()
    tree = ast.parse(src)
    ns = {"C": C}
    for node in tree.body:
        if isinstance(node, ast.ClassDef) and node.name in STRUCTS:
            mod = ast.Module(body=[node], type_ignores=[])
            exec(compile(mod, "rtlbl.py", "exec"), ns)
    return {k: ns[k] for k in STRUCTS}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_ctypes_layouts_match_the_header(tmp_path):
    classes = _binding_classes()
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rtlbl.h"', "int main(void) {"]
    for py, ct in STRUCTS.items():
        lines.append(f'  printf("{py} size %zu\\n", sizeof({ct}));')
        for name, _ in classes[py]._fields_:
            lines.append(f'  printf("{py} {name} %zu\\n", offsetof({ct}, {name}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        py, what, v = line.split()
        got[(py, what)] = int(v)
    for py, cls in classes.items():
        assert got[(py, "size")] == C.sizeof(cls), py
        for name, _ in cls._fields_:
            assert got[(py, name)] == getattr(cls, name).offset, (py, name)
