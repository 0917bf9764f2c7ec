"""Pins of the oracle's 16-point tabulated-profile kappa (the paper's own
formulation of Eq. (2)): at the reference state it is the plain Lorentz line
sum with an 8-point cutoff (the same 16 points, the same half width), away
from it each line scales with the cell's density and Eq. (1) ratio, and lines
near the grid's ends give their in-grid points."""
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from paper_cs_0703028_amd import inputs as I


def _grid(T, x=0.1, p=1.0, n=2):
    g = I.linear_T_grid(n, 0.1)
    g.T = np.full(g.n_cells, T, np.float64)
    g.x = np.full(g.n_cells, x, np.float64)
    g.p = np.full(g.n_cells, p, np.float64)
    return g


def test_reference_state_equals_plain_sum_with_8_point_cutoff():
    w = I.small_ragged()
    L = w.lines
    r = (L.nu - L.nu0) / L.dnu
    keep = (r - np.floor(r)) > 0        # centres on a grid point would get 17 plain points
    L = replace(L, nu=L.nu[keep], S=L.S[keep], gamma=L.gamma[keep], n_T=L.n_T[keep],
                E_lower=L.E_lower[keep])
    g = _grid(L.T_ref)                  # T = T_ref, p = 1 atm: gamma = gamma_ref, s = 1
    k16 = O.kappa_table16(g, L, [0, 3])
    kp = O.kappa(g, replace(L, cutoff=8 * L.dnu), [0, 3])
    assert np.allclose(k16, kp, rtol=1e-13, atol=0)
    assert np.count_nonzero(k16) > 0


def test_scales_with_density_and_strength_ratio():
    L = replace(I.small_ragged().lines, nu=np.array([1012.3456]), S=np.array([2e-21]),
                gamma=np.array([0.07]), n_T=np.array([0.5]), E_lower=np.array([800.0]))
    cold, hot = _grid(L.T_ref, 0.1, 1.0), _grid(1400.0, 0.2, 1.7)
    k0 = O.kappa_table16(cold, L, [0])[0]
    k1 = O.kappa_table16(hot, L, [0])[0]
    nz = k0 != 0
    assert np.count_nonzero(nz) == 16
    want = (O.density(1400.0, 0.2, 1.7) * O.strength_ratio(1400.0, L.T_ref, 1012.3456, 800.0)
            / (O.density(L.T_ref, 0.1, 1.0) * O.strength_ratio(L.T_ref, L.T_ref, 1012.3456, 800.0)))
    assert np.allclose(k1[nz] / k0[nz], want, rtol=1e-13)
    assert (k1[~nz] == 0).all()


def test_lines_at_the_grid_ends_keep_their_in_grid_points():
    base = I.small_ragged().lines
    L = replace(base, nu=np.array([base.nu0 - 0.033, base.nu0 + (base.n_nu - 1) * base.dnu + 0.041]),
                S=np.array([1e-21, 1e-21]), gamma=np.array([0.06, 0.06]), n_T=np.array([0.5, 0.5]),
                E_lower=None)
    k = O.kappa_table16(_grid(500.0), L, [0])[0]
    # centre at r = -3.3: m = -4, points -11..4 -> 0..4 in the grid
    assert np.count_nonzero(k[:10]) == 5 and k[5:10].sum() == 0
    # centre past the end: r = n_nu - 1 + 4.1, m = n_nu + 3, points n_nu - 4 ..
    assert np.count_nonzero(k[-10:]) == 4
