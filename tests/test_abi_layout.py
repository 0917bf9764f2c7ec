"""The Python binding agrees with include/rtlbl.h, as the C compiler reads
it (small C programs built with gcc against the header print the values):
* its ctypes mirrors of the public structs have the C layout: each struct's
  size and the offset of every field the binding names (a field added to
  the header but not to the binding, or in another place, changes a size or
  an offset; a field the header lacks fails to compile);
* its integer constants equal the header's enumerators and macros.
Host only."""
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


def _binding_constants():
    """The binding's top-level integer constants and its arithmetic-op codes,
    read from its source with literal evaluation only."""
    import ast
    src = open(os.path.join(ROOT, "paper_cs_0703028_amd", "rtlbl.py")).read()
    out = {}
    for node in ast.parse(src).body:
        if not isinstance(node, ast.Assign) or len(node.targets) != 1:
            continue
        tgt = node.targets[0]
        try:
            val = ast.literal_eval(node.value)
        except ValueError:
            continue
        if isinstance(tgt, ast.Name) and isinstance(val, int):
            out[tgt.id] = val
        elif isinstance(tgt, ast.Tuple) and isinstance(val, tuple):
            for e, v in zip(tgt.elts, val):
                out[e.id] = v
        elif isinstance(tgt, ast.Name) and tgt.id == "ARITH_OPS":
            for name, (code, _) in val.items():
                out["AR_" + name.upper()] = code
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_binding_constants_match_the_header(tmp_path):
    """Status codes, kappa modes, tally precisions, batch modes, the
    arithmetic-op codes and the two macros, as the header defines them."""
    consts = _binding_constants()
    # binding name -> header name
    names = {k: k for k in ("RT_OK", "RT_EINVAL", "RT_ENOMEM", "RT_EDEVICE", "RT_ESTATE",
                            "RT_EUNSUPPORTED", "RT_NO_DEVICE")}
    names.update({k: "RT_" + k for k in consts
                  if k.startswith(("KAPPA_", "TALLY_", "BATCH_", "AR_"))})
    names["ADAPTIVE_GROUP"] = "RT_ADAPTIVE_GROUP"
    lines = ["#include <stdio.h>", '#include "rtlbl.h"', "int main(void) {"]
    for py, h in names.items():
        lines.append(f'  printf("{py} %d\\n", (int)({h}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "consts.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "consts"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = dict((a, int(b)) for a, b in (line.split() for line in out.splitlines()))
    assert len(got) >= 30
    for py in names:
        assert got[py] == consts[py], py
