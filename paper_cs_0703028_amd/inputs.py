"""Seeded synthetic workloads for the line-by-line Monte-Carlo ray tracer.

The paper's real inputs (HITRAN-style H2O/CO2 line lists with millions of
lines, and the receptor's CFD temperature/pressure fields; Section 3) are not
available, so every workload is synthetic.  The laws below follow the
workload descriptions: Lorentz lines with uniform centres, log-normal
strengths (sigma = 2 around 1e-21 cm/molecule), uniform half widths
0.05-0.1 cm^-1 with temperature exponent 0.5, uniform lower-state energies
0-2000 cm^-1; cubic cells with a linear or Gaussian-hot-spot temperature
field.

This module is shared by the test-suite (which feeds the same inputs to the
FP64 oracle and to the HIP library) and by the benchmark.  It holds none of
the method's arithmetic: only draws from numpy's Philox4x64 bit generator,
keyed by (seed, stream), and the field definitions of the workloads.
Random numbers that the method itself draws (ray origins and directions) are
NOT made here.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

# Philox stream ids (second key word)
STREAM_CENTRES = 2
STREAM_STRENGTH = 3
STREAM_GAMMA = 4
STREAM_ELOWER = 5
STREAM_XH2O = 6
STREAM_CASES = 7
STREAM_TRAIN = 8
STREAM_INIT = 9
STREAM_CHECK = 10
STREAM_XGAS = 11   # mole fractions of further gases

T_REF = 296.0


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=np.array([seed, stream], dtype=np.uint64)))


@dataclass
class Grid:
    """nx*ny*nz cubic cells of edge cell_m [m]; cell c = ix + nx*(iy + ny*iz).
    T [K], x (H2O mole fraction), p [atm] per cell; T_wall [K] (0: cold)."""
    nx: int
    ny: int
    nz: int
    cell_m: float
    T: np.ndarray
    x: np.ndarray
    p: np.ndarray
    T_wall: float = 0.0

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz


@dataclass
class Lines:
    """Line list and spectral grid nu_j = nu0 + j*dnu, j < n_nu [cm^-1]."""
    nu: np.ndarray
    S: np.ndarray          # line strength at T_ref [cm/molecule]
    gamma: np.ndarray      # Lorentz HWHM at T_ref, 1 atm [cm^-1]
    n_T: np.ndarray        # temperature exponent of the half width
    E_lower: Optional[np.ndarray]  # lower-state energy [cm^-1] or None
    T_ref: float
    cutoff: float          # cm^-1
    nu0: float
    dnu: float
    n_nu: int


@dataclass
class Gas:
    """A further absorbing gas: mole fraction per cell and its line list (on
    the first gas's spectral grid)."""
    x: np.ndarray
    lines: Lines


@dataclass
class Workload:
    name: str
    grid: Grid
    lines: Lines
    n_rays: int
    seed: int = 0
    notes: dict = field(default_factory=dict)
    gases: tuple = ()   # further gases (Gas), summed into kappa by Eq. (2)


def line_list(n_lines: int, nu_lo: float, nu_hi: float, *, seed: int = 0,
              with_energy: bool = True, nu0: float = 1000.0, dnu: float = 0.01,
              n_nu: int = 10000, cutoff: float = 5.0, s_median: float = 1e-21,
              s_sigma: float = 2.0, gamma_lo: float = 0.05, gamma_hi: float = 0.1,
              n_exp: float = 0.5) -> Lines:
    nu = rng(seed, STREAM_CENTRES).uniform(nu_lo, nu_hi, n_lines)
    S = s_median * np.exp(s_sigma * rng(seed, STREAM_STRENGTH).standard_normal(n_lines))
    gamma = rng(seed, STREAM_GAMMA).uniform(gamma_lo, gamma_hi, n_lines)
    E = rng(seed, STREAM_ELOWER).uniform(0.0, 2000.0, n_lines) if with_energy else None
    return Lines(nu=nu, S=S, gamma=gamma, n_T=np.full(n_lines, n_exp), E_lower=E,
                 T_ref=T_REF, cutoff=cutoff, nu0=nu0, dnu=dnu, n_nu=n_nu)


def linear_T_grid(n: int, cell_m: float, T_lo: float = 300.0, T_hi: float = 1500.0,
                  x: float = 0.1, p: float = 1.0, T_wall: float = 0.0,
                  ny: Optional[int] = None, nz: Optional[int] = None) -> Grid:
    """T linear along x from T_lo (first cell) to T_hi (last cell)."""
    nx = n
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    ix = np.arange(nx * ny * nz) % nx
    T = T_lo + (T_hi - T_lo) * ix / max(nx - 1, 1)
    return Grid(nx, ny, nz, cell_m, T.astype(np.float64),
                np.full(nx * ny * nz, x), np.full(nx * ny * nz, p), T_wall)


def hot_spot_grid(n: int, length_m: float = 1.0, T_lo: float = 400.0, T_hi: float = 1800.0,
                  spread_m: float = 0.15, x_lo: float = 0.05, x_hi: float = 0.2,
                  seed: int = 0, T_wall: float = 0.0) -> Grid:
    """Gaussian hot spot at the domain centre; x_H2O uniform per cell."""
    h = length_m / n
    c = np.arange(n ** 3)
    ix, iy, iz = c % n, (c // n) % n, c // (n * n)
    centre = 0.5 * length_m
    r2 = ((ix + 0.5) * h - centre) ** 2 + ((iy + 0.5) * h - centre) ** 2 + \
        ((iz + 0.5) * h - centre) ** 2
    T = T_lo + (T_hi - T_lo) * np.exp(-r2 / (2.0 * spread_m ** 2))
    x = rng(seed, STREAM_XH2O).uniform(x_lo, x_hi, n ** 3)
    return Grid(n, n, n, h, T, x, np.ones(n ** 3), T_wall)


# ---------------------------------------------------------------- workloads
def plain_8cube(seed: int = 0) -> Workload:
    """8^3 cells of 0.125 m, T linear 300->1500 K, x = 0.1, p = 1 atm, 500
    lines in [1000, 1100] cm^-1, 10,000 points at 0.01 cm^-1, 1,024 rays."""
    g = linear_T_grid(8, 0.125)
    L = line_list(500, 1000.0, 1100.0, seed=seed, n_nu=10000)
    return Workload("plain_8cube_500lines_10k_nu_1024rays", g, L, 1024, seed)


def plain_32cube(seed: int = 0) -> Workload:
    """32^3 cells over 1 m, Gaussian hot spot 400-1800 K, x U[0.05,0.2],
    20,000 lines in [1000, 1500] cm^-1, 50,000 points, 2^20 rays."""
    g = hot_spot_grid(32, 1.0, seed=seed)
    L = line_list(20000, 1000.0, 1500.0, seed=seed, n_nu=50000)
    return Workload("plain_32cube_20k_lines_50k_nu_1M_rays", g, L, 1 << 20, seed)


def slab_1cell(seed: int = 0) -> Workload:
    """One 1 m cell at 1000 K, x = 0.1, p = 1 atm, black walls at 1500 K,
    the 8^3 workload's line list and spectral grid."""
    L = line_list(500, 1000.0, 1100.0, seed=seed, n_nu=10000)
    g = Grid(1, 1, 1, 1.0, np.array([1000.0]), np.array([0.1]), np.array([1.0]), 1500.0)
    return Workload("slab_1cell_1m_1000K_walls1500K", g, L, 1024, seed)


def small_ragged(seed: int = 3) -> Workload:
    """A non-cubic 5x6x7 grid with a ragged spectral length, for tests that
    must span several tiles and a partial tail quickly."""
    g = linear_T_grid(5, 0.1, ny=6, nz=7, T_lo=350.0, T_hi=1700.0, x=0.15, p=1.3)
    g.x = rng(seed, STREAM_XH2O).uniform(0.02, 0.3, g.n_cells)
    L = line_list(700, 995.0, 1040.0, seed=seed, n_nu=3037, nu0=1000.0)
    return Workload("small_ragged_5x6x7", g, L, 700, seed)


def batched_cases(n_cases: int = 64, seed: int = 0, sizes=(16, 24, 32, 48),
                  log2_rays=(14, 15, 16, 17, 18)) -> list:
    """Receiver cases: grid edge uniform in `sizes`, rays 2^k with k uniform
    in `log2_rays`, 1 m cube, hot-spot fields with per-case seeds; one shared
    list of 5,000 lines in [1000, 1200] cm^-1 on 20,000 points."""
    r = rng(seed, STREAM_CASES)
    L = line_list(5000, 1000.0, 1200.0, seed=seed, n_nu=20000)
    cases = []
    for k in range(n_cases):
        n = int(r.choice(sizes))
        nr = 1 << int(r.choice(log2_rays))
        g = hot_spot_grid(n, 1.0, seed=seed * 1000 + k + 1)
        cases.append(Workload(f"case{k}_{n}cube_{nr}rays", g, L, nr, seed * 1000 + k + 1))
    return cases


SURROGATE_BOX = (300.0, 2000.0, 0.01, 0.3, 0.5, 2.0)  # T, x_H2O, p ranges


def surrogate_samples(n: int = 1 << 16, seed: int = 0, box=SURROGATE_BOX):
    """Training gas states for the learned form: T, x_H2O, p uniform in the
    box (Philox stream 8)."""
    r = rng(seed, STREAM_TRAIN)
    T = r.uniform(box[0], box[1], n)
    x = r.uniform(box[2], box[3], n)
    p = r.uniform(box[4], box[5], n)
    return T, x, p


def with_lines(w: Workload, **kw) -> Workload:
    return replace(w, lines=replace(w.lines, **kw))


def spectral_shard_bounds(n_nu: int, n_shards: int, align: int) -> list:
    """Point ranges [lo, hi) of n_shards contiguous spectral shards, their
    boundaries on multiples of `align` points (the march chunk), so that no
    shard pads a chunk it shares with a neighbour."""
    units = -(-n_nu // align)
    cuts = [min(n_nu, (units * g // n_shards) * align) for g in range(n_shards + 1)]
    return [(cuts[g], cuts[g + 1]) for g in range(n_shards)]


def spectral_shard(w: Workload, lo: int, hi: int) -> Workload:
    """The workload on spectral points [lo, hi) of its grid only: the grid
    starts at point lo, and only the lines whose cutoff window can reach the
    range are kept (one GPU's share when a run is split by wavenumber)."""
    L = w.lines
    nu_lo = L.nu0 + lo * L.dnu
    nu_hi = L.nu0 + (hi - 1) * L.dnu
    margin = L.cutoff + L.dnu
    keep = (L.nu >= nu_lo - margin) & (L.nu <= nu_hi + margin)
    sub = replace(L, nu=L.nu[keep], S=L.S[keep], gamma=L.gamma[keep], n_T=L.n_T[keep],
                  E_lower=None if L.E_lower is None else L.E_lower[keep],
                  nu0=nu_lo, n_nu=hi - lo)
    return replace(w, name=f"{w.name}_points_{lo}_{hi}", lines=sub)


# A second, CO2-like absorber beside the first (H2O-like) one: its own line
# list drawn by the same laws from other streams (seed offset), weaker median
# strength and a steeper half-width temperature exponent, and its own mole
# fraction field.  The paper's Eq. (2) sums the gases; its listing pairs H2O
# with CO2.
GAS2_SEED_OFFSET = 1_000_003


def second_gas(w: Workload, n_lines: int, nu_lo: float, nu_hi: float, x_lo: float,
               x_hi: float) -> Workload:
    L = w.lines
    lines = line_list(n_lines, nu_lo, nu_hi, seed=w.seed + GAS2_SEED_OFFSET, nu0=L.nu0,
                      dnu=L.dnu, n_nu=L.n_nu, cutoff=L.cutoff, s_median=3e-22,
                      gamma_lo=0.06, gamma_hi=0.09, n_exp=0.75)
    x = rng(w.seed, STREAM_XGAS).uniform(x_lo, x_hi, w.grid.n_cells)
    return replace(w, name=w.name + "_plus_co2like", gases=w.gases + (Gas(x=x, lines=lines),))


def small_ragged_two_gases(seed: int = 3) -> Workload:
    return second_gas(small_ragged(seed), 300, 990.0, 1035.0, 0.01, 0.15)


def plain_8cube_two_gases(seed: int = 0) -> Workload:
    return second_gas(plain_8cube(seed), 200, 1000.0, 1100.0, 0.02, 0.1)


def plain_32cube_two_gases(seed: int = 0) -> Workload:
    return second_gas(plain_32cube(seed), 10000, 1000.0, 1500.0, 0.05, 0.15)
