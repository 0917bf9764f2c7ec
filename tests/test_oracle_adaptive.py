"""Pins of the oracle's adaptive line windows (the paper's announced next
version: points per line set by the local temperature and the line's
intensity).  Each is checked against something other than the windowed sum
itself: the plain oracle sum (vanishing tolerance, one isolated line), the
value criterion evaluated point by point in numpy from Eqs. (1)-(2), the
ordering of sums of non-negative terms, and the bound on what is dropped."""
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from paper_cs_0703028_amd import inputs as I

KB = 1.380649e-23                               # J/K (SI 2019, exact)
C2 = 6.62607015e-34 * 299792458.0 / KB * 100.0  # h c / k_B in cm K
ATM = 101325.0


def _one_line_lines(nu=1012.3456, S=2e-21, gamma=0.07, n_T=0.5, E=800.0):
    base = I.small_ragged().lines
    return replace(base, nu=np.array([nu]), S=np.array([S]), gamma=np.array([gamma]),
                   n_T=np.array([n_T]), E_lower=None if E is None else np.array([E]))


def _cells(T, x=0.1, p=1.0):
    T = np.atleast_1d(np.asarray(T, np.float64))
    g = I.linear_T_grid(len(T), 0.1, ny=1, nz=1)
    g.T = T.copy()
    g.x = np.broadcast_to(np.asarray(x, np.float64), T.shape).copy()
    g.p = np.broadcast_to(np.asarray(p, np.float64), T.shape).copy()
    return g


def _hard_count(lines):
    """Plain in-grid window points per line, from the integer window."""
    r = (lines.nu - lines.nu0) / lines.dnu
    m = np.floor(r)
    K = round(lines.cutoff / lines.dnu)
    lo = np.maximum(m - K + (r > m), 0)
    hi = np.minimum(m + K, lines.n_nu - 1)
    return np.maximum(hi - lo + 1, 0)


def test_vanishing_tolerance_is_the_plain_sum():
    w = I.small_ragged()
    cells = [0, 7, 8, 100, 209]
    ka = O.kappa_adaptive(w.grid, w.lines, 1e-300, cells)
    kp = O.kappa(w.grid, w.lines, cells)
    assert np.array_equal(ka, kp)
    assert O.adaptive_evals(w.grid, w.lines, 1e-300) == int(_hard_count(w.lines).sum()) * w.grid.n_cells


# one line alone sets its own reference level (its mass spread over the
# band), so only tolerances of a few percent and more cut its window
@pytest.mark.parametrize("T, E, eps", [(296.0, None, 0.1), (900.0, 800.0, 0.04),
                                       (1600.0, 1500.0, 0.5), (450.0, 100.0, 0.9)])
def test_isolated_line_keeps_points_at_or_above_threshold(T, E, eps):
    L = _one_line_lines(E=E)
    g = _cells(T, x=0.13, p=1.4)
    # one line: the band mean of the untruncated sum is u S s / (n_nu dnu)
    s = O.strength_ratio(T, L.T_ref, L.nu[0], 0.0 if E is None else E, E is not None)
    sbar = L.S[0] * s / (L.n_nu * L.dnu)
    assert O.mean_strength(T, L) == pytest.approx(sbar, rel=1e-15)
    thr = eps * O.density(T, 0.13, 1.4) * sbar
    kp = O.kappa(g, L, [0])[0]
    ka = O.kappa_adaptive(g, L, eps, [0])[0]
    clear = np.abs(kp / thr - 1) > 1e-9
    want = np.where(kp >= thr, kp, 0.0)
    assert np.array_equal(ka[clear], want[clear])
    kept = np.count_nonzero(ka)
    assert 0 < kept < np.count_nonzero(kp)


def test_mean_strength_counts_the_lines_that_meet_the_grid():
    L = _one_line_lines(E=None)
    K = L.cutoff / L.dnu
    top = L.nu0 + (L.n_nu - 1) * L.dnu
    inside = [L.nu0 - 0.5 * L.cutoff, top + 0.5 * L.cutoff]     # wings reach the grid
    outside = [L.nu0 - L.cutoff - 3 * L.dnu, top + L.cutoff + 3 * L.dnu]
    two = replace(L, nu=np.array(inside + outside), S=np.full(4, 1e-21), gamma=np.full(4, 0.07),
                  n_T=np.full(4, 0.5))
    assert K > 10
    assert O.mean_strength(500.0, two) == pytest.approx(2e-21 / (L.n_nu * L.dnu), rel=1e-15)


def test_group_window_is_the_union_of_its_cells_windows():
    L = _one_line_lines(E=600.0)
    T = np.linspace(300.0, 1700.0, 8)
    p = np.linspace(0.7, 1.6, 8)
    g8 = _cells(T, x=0.1, p=p)
    eps = 0.05
    grouped = O.kappa_adaptive(g8, L, eps)
    own = np.array([O.kappa_adaptive(_cells(T[c], 0.1, p[c]), L, eps, [0])[0] for c in range(8)])
    union = (own != 0).any(axis=0)
    for c in range(8):
        assert np.array_equal(grouped[c] != 0, union)
        assert (grouped[c] >= own[c]).all()
    # eight identical cells: the group window is the cell's own
    same = _cells(np.full(8, 800.0), 0.1, 1.2)
    alone = O.kappa_adaptive(_cells(800.0, 0.1, 1.2), L, eps, [0])[0]
    assert np.array_equal(O.kappa_adaptive(same, L, eps, [5])[0], alone)
    # one line: the windows are nested, the union is the widest cell's own
    counts = [np.count_nonzero(k) for k in own]
    assert np.count_nonzero(union) == max(counts) > min(counts)


def test_nested_in_the_tolerance_and_below_the_plain_sum():
    w = I.small_ragged()
    cells = [3, 64, 150]
    kp = O.kappa(w.grid, w.lines, cells)
    prev = kp
    counts = []
    for eps in (1e-6, 1e-4, 1e-2):
        ka = O.kappa_adaptive(w.grid, w.lines, eps, cells)
        assert (ka <= prev).all() and (ka >= 0).all()
        counts.append(O.adaptive_evals(w.grid, w.lines, eps))
        prev = ka
    assert counts[0] > counts[1] > counts[2] > 0


def test_dropped_remainder_within_its_bound():
    w = I.small_ragged()
    L, g = w.lines, w.grid
    cells = [0, 41, 133, 209]
    eps = 1e-4
    kp = O.kappa(g, L, cells)
    ka = O.kappa_adaptive(g, L, eps, cells)
    r = (L.nu - L.nu0) / L.dnu
    K = round(L.cutoff / L.dnu)
    j = np.arange(L.n_nu)
    n_lines_at = ((np.abs(j[:, None] - r[None, :]) <= K)).sum(axis=1)
    for row, c in enumerate(cells):
        kbar = O.density(g.T[c], g.x[c], g.p[c]) * O.mean_strength(g.T[c], L)
        gap = kp[row] - ka[row]
        assert (gap >= 0).all()
        assert (gap <= n_lines_at * eps * kbar * (1 + 1e-12)).all()
        assert gap.max() > 0


def _numpy_values(g, L, c):
    """Per (line, point) Lorentz values of cell c and its threshold factor,
    written from Eqs. (1)-(2) in numpy: rows of lines, columns of points."""
    T, x, p = g.T[c], g.x[c], g.p[c]
    u = x * p * ATM / (KB * T) * 1e-6
    s = ((L.T_ref / T) ** 1.5 * np.exp(-C2 * L.E_lower * (1 / T - 1 / L.T_ref))
         * (1 - np.exp(-C2 * L.nu / T)) / (1 - np.exp(-C2 * L.nu / L.T_ref)))
    gam = L.gamma * p * (L.T_ref / T) ** L.n_T
    r = (L.nu - L.nu0) / L.dnu
    K = round(L.cutoff / L.dnu)
    meets = (r >= -K) & (r <= L.n_nu - 1 + K)
    sbar = (L.S * s)[meets].sum() / (L.n_nu * L.dnu)
    d = (np.arange(L.n_nu)[None, :] - r[:, None]) * L.dnu
    v = u * L.S[:, None] * s[:, None] * gam[:, None] / (np.pi * (d * d + gam[:, None] ** 2))
    hard = np.abs(np.arange(L.n_nu)[None, :] - r[:, None]) <= K
    return v, hard, u * sbar


def test_brute_force_value_criterion_counts_and_sums():
    g = I.linear_T_grid(2, 0.1, ny=2, nz=3, T_lo=350.0, T_hi=1650.0)
    g.x = I.rng(5, I.STREAM_XH2O).uniform(0.02, 0.3, g.n_cells)
    g.p = np.linspace(0.8, 1.5, g.n_cells)
    g.T = np.linspace(350.0, 1650.0, g.n_cells)[::-1].copy()
    L = I.line_list(60, 998.0, 1005.0, seed=9, nu0=1000.0, dnu=0.01, n_nu=400, cutoff=1.0)
    eps = 2e-4
    per = [_numpy_values(g, L, c) for c in range(g.n_cells)]
    total = 0
    ambiguous = 0
    ka = O.kappa_adaptive(g, L, eps)
    for c in range(g.n_cells):
        grp = range(8 * (c // 8), min(g.n_cells, 8 * (c // 8) + 8))
        hits = np.zeros_like(per[c][1])
        for q in grp:
            v, hard, kbar = per[q]
            thr = eps * kbar
            hits |= hard & (v >= thr)
            ambiguous += int((hard & (np.abs(v / thr - 1) < 1e-9)).sum())
        total += int(hits.sum())
        want = np.where(hits, per[c][0], 0.0).sum(axis=0)
        assert np.allclose(ka[c], want, rtol=1e-11, atol=1e-300)
    got = O.adaptive_evals(g, L, eps)
    assert abs(got - total) <= ambiguous
    assert 0 < total < sum(int(p[1].sum()) for p in per)


def test_zero_strengths_keep_the_plain_window():
    # sbar = 0: no reference level, the hard window is kept (and every term is 0)
    w = I.small_ragged()
    Z = replace(w.lines, S=np.zeros_like(w.lines.S))
    assert O.mean_strength(900.0, Z) == 0.0
    assert O.adaptive_evals(w.grid, Z, 1e-3) == int(_hard_count(Z).sum()) * w.grid.n_cells
    assert not O.kappa_adaptive(w.grid, Z, 1e-3, [0, 100]).any()
    # a zero-strength line among others keeps no point
    L = w.lines
    one = replace(L, nu=L.nu[:1], S=np.zeros(1), gamma=L.gamma[:1], n_T=L.n_T[:1],
                  E_lower=L.E_lower[:1])
    both = replace(L, nu=L.nu[:2], S=np.array([0.0, L.S[1]]), gamma=L.gamma[:2], n_T=L.n_T[:2],
                   E_lower=L.E_lower[:2])
    second = replace(L, nu=L.nu[1:2], S=L.S[1:2], gamma=L.gamma[1:2], n_T=L.n_T[1:2],
                     E_lower=L.E_lower[1:2])
    assert O.adaptive_evals(w.grid, both, 0.05) == O.adaptive_evals(w.grid, second, 0.05)
    assert O.adaptive_evals(w.grid, one, 0.05) == int(_hard_count(one).sum()) * w.grid.n_cells
