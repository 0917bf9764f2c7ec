"""The FP64 oracle's march spread over host threads, for parity tests whose
ray counts would take the single-threaded oracle minutes.

Test infrastructure: every number still comes from ``oracle/rt_oracle.c``.
The rays are split into contiguous slices, each slice is marched by the
oracle on its own thread (ctypes releases the interpreter lock), and the
slices' FP64 tallies are added in slice order.  Only the order of the FP64
additions of the tallies differs from one oracle call over all rays (a
relative difference of order 1e-15)."""
from __future__ import annotations

import concurrent.futures as cf
import os

import numpy as np

from oracle import oracle as O


def threads() -> int:
    """Host threads for the pool: the OpenMP count the oracle sees, at most 16."""
    return max(1, min(16, O.num_threads(), os.cpu_count() or 1))


def march(grid, lines, Os, Ds, weight, kap, B, cell_row=None, n_threads=None):
    n_threads = n_threads or threads()
    n = Os.shape[0]
    bounds = np.linspace(0, n, n_threads + 1).astype(int)
    parts = [(bounds[k], bounds[k + 1]) for k in range(n_threads) if bounds[k + 1] > bounds[k]]

    def one(p):
        a, b = p
        return O.march(grid, lines, Os[a:b], Ds[a:b], weight, kap, B, cell_row=cell_row)[:3]

    with cf.ThreadPoolExecutor(max_workers=len(parts)) as ex:
        res = list(ex.map(one, parts))
    absorbed = np.zeros(grid.n_cells)
    emitted = np.zeros(grid.n_cells)
    balance = np.zeros(4)
    for a, e, b in res:
        absorbed += a
        emitted += e
        balance += b
    return absorbed, emitted, balance


def run(grid, lines, n_rays_total, seed=0, begin=0, count=None, n_threads=None):
    """Kappa and Planck rows of every cell (the oracle's OpenMP loops), then
    the pooled march of rays [begin, begin + count) of n_rays_total."""
    if count is None:
        count = n_rays_total - begin
    Os, Ds, _ = O.rays(seed, begin, count, grid.nx, grid.ny, grid.nz)
    kap = O.kappa(grid, lines)
    B = O.planck_rows(grid, lines)
    w = O.ray_weight(grid, lines, n_rays_total)
    a, e, bal = march(grid, lines, Os, Ds, w, kap, B, n_threads=n_threads)
    return dict(absorbed=a, emitted=e, balance=bal, kappa=kap, planck=B)
