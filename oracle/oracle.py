"""ctypes front end of the FP64 CPU oracle (``rt_oracle.c``).

Test infrastructure only: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the library product never does.
Nothing here performs any of the method's arithmetic -- every number comes from
``rt_oracle.c``; this file only marshals numpy arrays in and out -- except the
outer sum over gases of Eq. (2) in ``kappa_gases``, a plain FP64 addition of
the per-gas line sums in gas order.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rt_oracle.c")
_LIB = os.path.join(_HERE, "librt_oracle.so")

_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, -O2, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-std=gnu11", "-O2", "-fopenmp", "-ffp-contract=off",
            "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.orc_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
        L.orc_philox4x64_10.restype = None
        L.orc_ray.argtypes = [C.c_uint64, C.c_uint64, C.c_int, C.c_int, C.c_int,
                              _i64p, _i64p, C.POINTER(C.c_int32)]
        L.orc_ray.restype = C.c_int
        L.orc_segments.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, _i64p, _i64p,
                                   _i32p, _f64p, C.c_int]
        L.orc_segments.restype = C.c_int
        L.orc_density.argtypes = [C.c_double] * 3
        L.orc_density.restype = C.c_double
        L.orc_strength_ratio.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int]
        L.orc_strength_ratio.restype = C.c_double
        L.orc_half_width.argtypes = [C.c_double] * 5
        L.orc_half_width.restype = C.c_double
        L.orc_kappa.argtypes = [C.c_int, _i32p, _f64p, _f64p, _f64p, C.c_int,
                                _f64p, _f64p, _f64p, _f64p, C.c_void_p, C.c_double,
                                C.c_double, C.c_double, C.c_double, C.c_int, _f64p]
        L.orc_kappa.restype = C.c_int
        L.orc_kappa_table16.argtypes = [C.c_int, _i32p, _f64p, _f64p, _f64p, C.c_int,
                                        _f64p, _f64p, _f64p, C.c_void_p, C.c_double,
                                        C.c_double, C.c_double, C.c_int, _f64p]
        L.orc_kappa_table16.restype = C.c_int
        L.orc_mean_strength.argtypes = [C.c_double, C.c_int, _f64p, _f64p, C.c_void_p,
                                        C.c_double, C.c_double, C.c_double, C.c_double,
                                        C.c_int]
        L.orc_mean_strength.restype = C.c_double
        L.orc_kappa_adaptive.argtypes = [C.c_int, _i32p, C.c_int, _f64p, _f64p, _f64p, C.c_int,
                                         _f64p, _f64p, _f64p, _f64p, C.c_void_p, C.c_double,
                                         C.c_double, C.c_double, C.c_double, C.c_int,
                                         C.c_double, C.c_int, _f64p]
        L.orc_kappa_adaptive.restype = C.c_int
        L.orc_wing_return.argtypes = L.orc_kappa_adaptive.argtypes
        L.orc_wing_return.restype = C.c_int
        L.orc_adaptive_evals.argtypes = [C.c_int, _f64p, _f64p, C.c_int, _f64p, _f64p, _f64p,
                                         _f64p, C.c_void_p, C.c_double, C.c_double, C.c_double,
                                         C.c_double, C.c_int, C.c_double, C.c_int]
        L.orc_adaptive_evals.restype = C.c_double
        L.orc_planck.argtypes = [C.c_double, C.c_double]
        L.orc_planck.restype = C.c_double
        L.orc_planck_rows.argtypes = [C.c_int, _i32p, _f64p, C.c_double, C.c_double,
                                      C.c_int, _f64p]
        L.orc_planck_rows.restype = C.c_int
        L.orc_march.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, _i64p, _i64p,
                                C.c_double, C.c_double, C.c_double, C.c_double, C.c_int,
                                _f64p, _f64p, C.c_void_p, _f64p, _f64p, _f64p, C.c_void_p]
        L.orc_march.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_set_num_threads.restype = None
        L.orc_boundary_area.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double]
        L.orc_boundary_area.restype = C.c_double
        for name in ("orc_const_c1", "orc_const_c2"):
            getattr(L, name).restype = C.c_double
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the OpenMP loops over cells (a timing control only)."""
    lib().orc_set_num_threads(int(n))


def c1() -> float:
    return lib().orc_const_c1()


def c2() -> float:
    return lib().orc_const_c2()


def philox(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(np.ascontiguousarray(ctr, np.uint64),
                            np.ascontiguousarray(key, np.uint64), out)
    return out


def ray(seed: int, r: int, nx: int, ny: int, nz: int):
    O = np.zeros(3, np.int64)
    D = np.zeros(3, np.int64)
    f = C.c_int32(0)
    lib().orc_ray(seed, r, nx, ny, nz, O, D, C.byref(f))
    return O, D, int(f.value)


def rays(seed: int, begin: int, count: int, nx: int, ny: int, nz: int):
    """Origins, directions and faces of rays begin .. begin+count-1."""
    O = np.zeros((count, 3), np.int64)
    D = np.zeros((count, 3), np.int64)
    F = np.zeros(count, np.int32)
    for k in range(count):
        O[k], D[k], F[k] = ray(seed, begin + k, nx, ny, nz)
    return O, D, F


def segments(nx, ny, nz, h_cm, O, D):
    cap = nx + ny + nz + 3
    cells = np.zeros(cap, np.int32)
    lens = np.zeros(cap, np.float64)
    n = lib().orc_segments(nx, ny, nz, h_cm, np.ascontiguousarray(O, np.int64),
                           np.ascontiguousarray(D, np.int64), cells, lens, cap)
    if n < 0:
        raise RuntimeError(f"orc_segments failed ({n})")
    return cells[:n].copy(), lens[:n].copy()


def density(T, x, p):
    return lib().orc_density(T, x, p)


def strength_ratio(T, T_ref, nu, E, have_E=True):
    return lib().orc_strength_ratio(T, T_ref, nu, E, int(have_E))


def half_width(g, n, T, T_ref, p):
    return lib().orc_half_width(g, n, T, T_ref, p)


def kappa(grid, lines, cell_list=None) -> np.ndarray:
    """kappa rows [len(cell_list)][n_nu] in cm^-1 (all cells if None)."""
    if cell_list is None:
        cell_list = np.arange(grid.n_cells, dtype=np.int32)
    cell_list = np.ascontiguousarray(cell_list, np.int32)
    out = np.zeros((len(cell_list), lines.n_nu), np.float64)
    E = lines.E_lower
    Ep = None if E is None else np.ascontiguousarray(E, np.float64).ctypes.data_as(C.c_void_p)
    rc = lib().orc_kappa(len(cell_list), cell_list, _f(grid.T), _f(grid.x), _f(grid.p),
                         len(lines.nu), _f(lines.nu), _f(lines.S), _f(lines.gamma),
                         _f(lines.n_T), Ep, lines.T_ref, lines.cutoff, lines.nu0,
                         lines.dnu, lines.n_nu, out)
    if rc != 0:
        raise ValueError("cutoff/dnu is not an integer")
    return out


def kappa_table16(grid, lines, cell_list=None) -> np.ndarray:
    """The paper's 16-point tabulated-profile kappa rows (rt_oracle.c)."""
    if cell_list is None:
        cell_list = np.arange(grid.n_cells, dtype=np.int32)
    cell_list = np.ascontiguousarray(cell_list, np.int32)
    out = np.zeros((len(cell_list), lines.n_nu), np.float64)
    E = lines.E_lower
    Ep = None if E is None else np.ascontiguousarray(E, np.float64).ctypes.data_as(C.c_void_p)
    lib().orc_kappa_table16(len(cell_list), cell_list, _f(grid.T), _f(grid.x), _f(grid.p),
                            len(lines.nu), _f(lines.nu), _f(lines.S), _f(lines.gamma), Ep,
                            lines.T_ref, lines.nu0, lines.dnu, lines.n_nu, out)
    return out


ADAPTIVE_GROUP = 8   # cells sharing one line window in the adaptive form


def mean_strength(T, lines) -> float:
    """sbar = sum_i S_i s_i(T) / (n_nu dnu) over the lines meeting the grid:
    the band-mean kappa of a cell divided by its density u."""
    E = None if lines.E_lower is None else np.ascontiguousarray(lines.E_lower, np.float64)
    Ep = None if E is None else E.ctypes.data_as(C.c_void_p)
    return lib().orc_mean_strength(T, len(lines.nu), _f(lines.nu), _f(lines.S), Ep,
                                   lines.T_ref, lines.cutoff, lines.nu0, lines.dnu, lines.n_nu)


def kappa_adaptive(grid, lines, eps, cell_list=None, group=ADAPTIVE_GROUP,
                   wings=False) -> np.ndarray:
    """kappa rows of the adaptive-window form (rt_oracle.c); with wings, each
    row also carries its cell's wing-return constant (wing_return)."""
    if cell_list is None:
        cell_list = np.arange(grid.n_cells, dtype=np.int32)
    cell_list = np.ascontiguousarray(cell_list, np.int32)
    out = np.zeros((len(cell_list), lines.n_nu), np.float64)
    args, keep = _adaptive_args(grid, lines, eps, cell_list, group)
    rc = lib().orc_kappa_adaptive(*args, out)
    if rc != 0:
        raise ValueError(f"orc_kappa_adaptive: bad arguments ({rc})")
    if wings:
        out += wing_return(grid, lines, eps, cell_list, group)[:, None]
    return out


def wing_return(grid, lines, eps, cell_list=None, group=ADAPTIVE_GROUP) -> np.ndarray:
    """Per listed cell, the band-uniform constant that returns the Lorentz
    mass of the points the adaptive windows drop (rt_oracle.c)."""
    if cell_list is None:
        cell_list = np.arange(grid.n_cells, dtype=np.int32)
    cell_list = np.ascontiguousarray(cell_list, np.int32)
    out = np.zeros(len(cell_list), np.float64)
    args, keep = _adaptive_args(grid, lines, eps, cell_list, group)
    rc = lib().orc_wing_return(*args, out)
    if rc != 0:
        raise ValueError(f"orc_wing_return: bad arguments ({rc})")
    return out


def _adaptive_args(grid, lines, eps, cell_list, group):
    # the arguments, and the energies array that the raw pointer in them
    # refers to (the caller keeps it alive over the call)
    E = None if lines.E_lower is None else np.ascontiguousarray(lines.E_lower, np.float64)
    Ep = None if E is None else E.ctypes.data_as(C.c_void_p)
    return (len(cell_list), cell_list, grid.n_cells, _f(grid.T), _f(grid.x), _f(grid.p),
            len(lines.nu), _f(lines.nu), _f(lines.S), _f(lines.gamma), _f(lines.n_T), Ep,
            lines.T_ref, lines.cutoff, lines.nu0, lines.dnu, lines.n_nu, float(eps),
            int(group)), E


def adaptive_evals(grid, lines, eps, group=ADAPTIVE_GROUP) -> int:
    """(cell, line, point) evaluations the adaptive form keeps on the grid."""
    E = None if lines.E_lower is None else np.ascontiguousarray(lines.E_lower, np.float64)
    Ep = None if E is None else E.ctypes.data_as(C.c_void_p)
    v = lib().orc_adaptive_evals(grid.n_cells, _f(grid.T), _f(grid.p), len(lines.nu),
                                 _f(lines.nu), _f(lines.S), _f(lines.gamma), _f(lines.n_T), Ep,
                                 lines.T_ref, lines.cutoff, lines.nu0, lines.dnu, lines.n_nu,
                                 float(eps), int(group))
    if v < 0:
        raise ValueError(f"orc_adaptive_evals: bad arguments ({v})")
    return int(v)


def kappa_gases(grid, lines, gases=(), cell_list=None) -> np.ndarray:
    """Eq. (2) with its outer sum over gases: gas 0 is (grid.x, lines); each
    further gas (an object with .x per cell and .lines on the same spectral
    grid) adds its own line sum at its own mole fraction."""
    total = kappa(grid, lines, cell_list)
    for g in gases:
        L = g.lines
        if (L.nu0, L.dnu, L.n_nu, L.cutoff, L.T_ref) != (lines.nu0, lines.dnu, lines.n_nu,
                                                        lines.cutoff, lines.T_ref):
            raise ValueError("every gas must use the first gas's spectral grid, cutoff and T_ref")
        total = total + kappa(replace(grid, x=np.asarray(g.x, np.float64)), L, cell_list)
    return total


def planck(nu, T) -> float:
    return lib().orc_planck(nu, T)


def planck_rows(grid, lines, cell_list=None) -> np.ndarray:
    if cell_list is None:
        cell_list = np.arange(grid.n_cells, dtype=np.int32)
    cell_list = np.ascontiguousarray(cell_list, np.int32)
    out = np.zeros((len(cell_list), lines.n_nu), np.float64)
    lib().orc_planck_rows(len(cell_list), cell_list, _f(grid.T), lines.nu0, lines.dnu,
                          lines.n_nu, out)
    return out


def boundary_area(nx, ny, nz, h_m):
    return lib().orc_boundary_area(nx, ny, nz, h_m)


def march(grid, lines, O, D, weight, kap, B, cell_row=None, want_exit=False):
    """Absorbed/emitted power per cell [W], balance (entering, emitted,
    absorbed, escaped) [W] and optionally exit intensity per (ray, j)."""
    O = np.ascontiguousarray(O, np.int64).reshape(-1, 3)
    D = np.ascontiguousarray(D, np.int64).reshape(-1, 3)
    n_rays = O.shape[0]
    absorbed = np.zeros(grid.n_cells, np.float64)
    emitted = np.zeros(grid.n_cells, np.float64)
    balance = np.zeros(4, np.float64)
    exit_I = np.zeros((n_rays, lines.n_nu), np.float64) if want_exit else None
    cr = None
    if cell_row is not None:
        cell_row = np.ascontiguousarray(cell_row, np.int32)
        cr = cell_row.ctypes.data_as(C.c_void_p)
    ep = exit_I.ctypes.data_as(C.c_void_p) if want_exit else None
    rc = lib().orc_march(grid.nx, grid.ny, grid.nz, grid.cell_m * 100.0, n_rays, O, D,
                         weight, grid.T_wall, lines.nu0, lines.dnu, lines.n_nu,
                         _f(kap), _f(B), cr, absorbed, emitted, balance, ep)
    if rc != 0:
        raise RuntimeError(f"orc_march failed ({rc})")
    return absorbed, emitted, balance, exit_I


def ray_weight(grid, lines, n_rays_total):
    """w = pi * A_boundary * dnu / N_rays (W per unit radiance)."""
    return np.pi * boundary_area(grid.nx, grid.ny, grid.nz, grid.cell_m) * lines.dnu / n_rays_total


def run(grid, lines, n_rays_total, seed=0, begin=0, count=None, cells_needed_only=False):
    """Whole path on the CPU: kappa, Planck, Philox rays, march, tally."""
    if count is None:
        count = n_rays_total - begin
    O, D, _ = rays(seed, begin, count, grid.nx, grid.ny, grid.nz)
    h_cm = grid.cell_m * 100.0
    if cells_needed_only:
        visited = set()
        for k in range(count):
            c, _ = segments(grid.nx, grid.ny, grid.nz, h_cm, O[k], D[k])
            visited.update(int(v) for v in c)
        cell_list = np.array(sorted(visited), np.int32)
    else:
        cell_list = np.arange(grid.n_cells, dtype=np.int32)
    kap = kappa(grid, lines, cell_list)
    B = planck_rows(grid, lines, cell_list)
    row = np.full(grid.n_cells, -1, np.int32)
    row[cell_list] = np.arange(len(cell_list), dtype=np.int32)
    w = ray_weight(grid, lines, n_rays_total)
    a, e, bal, _ = march(grid, lines, O, D, w, kap, B, cell_row=row)
    return dict(absorbed=a, emitted=e, balance=bal, cell_list=cell_list, kappa=kap, planck=B)


def _f(a):
    return np.ascontiguousarray(a, np.float64)
