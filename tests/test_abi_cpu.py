"""Host-side checks of the C ABI that need no GPU: the shared library loads and
exports every entry point the public header declares, the Python binding names
the same set, and a host-only handle (RT_NO_DEVICE) runs the library's own
argument and call-order checks."""
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


# --------------------------------------------------------- host-only handles
# A handle created with RT_NO_DEVICE runs the library's argument and
# call-order checks without a GPU: the same RT_EINVAL / RT_ESTATE results a
# device handle gives, and RT_EUNSUPPORTED where a call would need a device.

@pytest.fixture()
def rt():
    if not os.path.exists(LIB):
        pytest.skip("librtlbl.so not built")
    from paper_cs_0703028_amd import rtlbl
    return rtlbl


@pytest.fixture()
def host(rt):
    t = rt.Tracer.host_only()
    yield t
    t.close()


def _status(rt, fn):
    try:
        fn()
    except rt.RtError as e:
        return e.status
    return rt.RT_OK


def test_host_only_grid_checks(rt, host):
    from paper_cs_0703028_amd import inputs as I
    g = I.small_ragged().grid
    assert _status(rt, lambda: host.setup_grid(g)) == rt.RT_OK
    for field, k, v, word in (("T", 3, -1.0, "T"), ("T", 0, float("nan"), "finite"),
                              ("x", 5, 1.5, "x_h2o"), ("p", 7, 0.0, "p")):
        bad = I.small_ragged().grid
        arr = getattr(bad, field).copy()
        arr[k] = v
        setattr(bad, field, arr)
        assert _status(rt, lambda: host.setup_grid(bad)) == rt.RT_EINVAL
        assert word in host.last_error(), host.last_error()
    import numpy as np
    one = np.ones(1)
    f = rt.lib.rt_setup_grid
    assert f(host._h, 0, 1, 1, 0.1, one, one, one, 0.0) == rt.RT_EINVAL
    assert f(host._h, (1 << 20) + 1, 1, 1, 0.1, one, one, one, 0.0) == rt.RT_EINVAL
    big = 1 << 11   # 2^33 cells: refused before the arrays are read
    assert f(host._h, big, big, big, 0.1, one, one, one, 0.0) == rt.RT_EINVAL
    assert "2^31" in host.last_error()
    assert f(host._h, 1, 1, 1, -0.1, one, one, one, 0.0) == rt.RT_EINVAL
    assert f(host._h, 1, 1, 1, 0.1, one, one, one, -5.0) == rt.RT_EINVAL


def test_host_only_line_checks(rt, host):
    from dataclasses import replace
    from paper_cs_0703028_amd import inputs as I
    w = I.small_ragged()
    L = w.lines
    ok = lambda lines: _status(rt, lambda: host.setup_lines(lines))
    assert ok(L) == rt.RT_OK
    assert host.required_pitch() % rt.MARCH_CHUNK == 0
    assert host.required_pitch() >= L.n_nu
    assert ok(replace(L, cutoff=5.005)) == rt.RT_EINVAL and "integer" in host.last_error()
    assert ok(replace(L, n_nu=0)) == rt.RT_EINVAL
    assert ok(replace(L, dnu=-0.01)) == rt.RT_EINVAL
    assert ok(replace(L, T_ref=0.0)) == rt.RT_EINVAL
    assert ok(replace(L, n_nu=1 << 24)) == rt.RT_EINVAL and "2^24" in host.last_error()
    for field, v, word in (("S", -1e-21, "S_ref"), ("gamma", 0.0, "gamma"),
                           ("E_lower", -1.0, "E_lower"), ("nu", float("inf"), "finite")):
        arr = getattr(L, field).copy()
        arr[2] = v
        assert ok(replace(L, **{field: arr})) == rt.RT_EINVAL
        assert word in host.last_error(), host.last_error()


def test_host_only_call_order(rt, host):
    from paper_cs_0703028_amd import inputs as I
    w = I.small_ragged()
    h = host._h
    lib = rt.lib
    # before any setup
    assert lib.rt_compute_kappa(h, 0, None, None, 1536) == rt.RT_ESTATE
    assert lib.rt_trace_rays(h, 0, 10, 0, 10, 0) == rt.RT_ESTATE
    assert lib.rt_tally(h, None, None, None) == rt.RT_ESTATE
    assert lib.rt_required_pitch(h) == -1
    host.setup_grid(w.grid)
    assert lib.rt_compute_kappa(h, 0, None, None, 1536) == rt.RT_ESTATE   # no lines yet
    assert _status(rt, lambda: host.setup_gas(1, None)) == rt.RT_ESTATE          # no lines yet
    host.setup_lines(w.lines)
    ld = host.required_pitch()
    fake = ctypes.c_void_p(1 << 20)             # never dereferenced by the checks
    assert lib.rt_compute_kappa(h, 9, fake, None, ld) == rt.RT_EINVAL            # mode
    assert lib.rt_compute_kappa(h, 0, None, None, ld) == rt.RT_EINVAL            # NULL table
    assert lib.rt_compute_kappa(h, 0, fake, None, ld - 1) == rt.RT_EINVAL        # pitch
    assert lib.rt_compute_kappa(h, 0, ctypes.c_void_p((1 << 20) + 4), None, ld) == rt.RT_EINVAL
    assert lib.rt_compute_kappa(h, rt.KAPPA_ADAPTIVE, fake, None, ld) == rt.RT_ESTATE  # no eps
    assert lib.rt_compute_kappa(h, rt.KAPPA_SURROGATE, fake, None, ld) == rt.RT_ESTATE
    assert lib.rt_set_line_tolerance(h, 0.0) == rt.RT_EINVAL
    assert lib.rt_set_line_tolerance(h, 1e-4) == rt.RT_OK
    # every check passed: the work itself needs a device
    assert lib.rt_compute_kappa(h, 0, fake, None, ld) == rt.RT_EUNSUPPORTED
    assert "host-only" in host.last_error()
    assert lib.rt_trace_rays(h, 0, 10, 0, 10, 0) == rt.RT_ESTATE               # no kappa
    assert lib.rt_trace_rays_noalloc(h, 0, 10, 0, 10, 0) == rt.RT_ESTATE
    assert lib.rt_tally(h, None, None, None) == rt.RT_EUNSUPPORTED
    assert lib.rt_reset_tally(h) == rt.RT_EUNSUPPORTED


def test_host_only_surrogate_calls(rt, host):
    """Phase timing is a host-side switch (no device, no trained network
    needed); the other learned-form calls still report what they lack."""
    from paper_cs_0703028_amd import inputs as I
    lib = rt.lib
    h = host._h
    assert lib.rt_surrogate_time_phases(None, 1) == rt.RT_EINVAL
    assert lib.rt_surrogate_time_phases(h, 1) == rt.RT_OK
    assert lib.rt_surrogate_time_phases(h, 0) == rt.RT_OK
    st = rt.SurrogateStats()
    assert lib.rt_surrogate_get_stats(h, ctypes.byref(st)) == rt.RT_ESTATE   # nothing trained
    w = I.small_ragged()
    host.setup_grid(w.grid)
    host.setup_lines(w.lines)
    ld = host.required_pitch()
    fake = ctypes.c_void_p(1 << 20)
    assert lib.rt_compute_kappa(h, rt.KAPPA_SURROGATE, fake, None, ld) == rt.RT_ESTATE


def test_host_only_batch_checks(rt, host):
    from dataclasses import replace
    from paper_cs_0703028_amd import inputs as I
    cases = I.batched_cases(4)
    assert _status(rt, lambda: host.batch_workspace_size(cases)) == rt.RT_ESTATE  # no lines
    host.setup_lines(cases[0].lines)
    assert host.batch_workspace_size(cases) > 0
    tun = rt.Tracer.default_tuning()
    tun.chunk_points = 1000                     # not a multiple of the march chunk
    assert _status(rt, lambda: host.batch_workspace_size(cases, tun)) == rt.RT_EINVAL
    tun = rt.Tracer.default_tuning()
    tun.mode = 2                                # no such launch shape
    assert _status(rt, lambda: host.batch_workspace_size(cases, tun)) == rt.RT_EINVAL
    tun = rt.Tracer.default_tuning()
    tun.slots = 1                               # the persistent queue needs two slabs
    tun.slots = 9
    assert _status(rt, lambda: host.batch_workspace_size(cases, tun)) == rt.RT_EINVAL
    tun.slots = 1
    assert tun.mode == rt.BATCH_CHUNKED and host.batch_workspace_size(cases, tun) > 0
    tun.mode = rt.BATCH_PERSISTENT
    assert _status(rt, lambda: host.batch_workspace_size(cases, tun)) == rt.RT_EINVAL
    # two slabs each, chunked: over the cells of every case; persistent: of
    # the largest case
    ch, pe = rt.Tracer.default_tuning(), rt.Tracer.default_tuning()
    ch.slots = 2
    pe.mode, pe.slots = rt.BATCH_PERSISTENT, 2
    cells = [c.grid.n_cells for c in cases]
    grow = 2 * (sum(cells) - max(cells)) * ch.chunk_points * 4
    diff = host.batch_workspace_size(cases, ch) - host.batch_workspace_size(cases, pe)
    assert abs(diff - grow) < 1 << 16, (diff, grow)
    bad = replace(cases[1], n_rays=0)
    assert _status(rt, lambda: host.batch_workspace_size([cases[0], bad])) == rt.RT_EINVAL
    g = I.hot_spot_grid(16, 1.0, seed=3)
    g.T = g.T.copy()
    g.T[0] = 0.0
    assert _status(rt, lambda: host.batch_workspace_size([replace(cases[0], grid=g)])) \
        == rt.RT_EINVAL
    assert _status(rt, lambda: host.batch_run(cases)) == rt.RT_EUNSUPPORTED
