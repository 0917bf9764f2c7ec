"""Pins of the oracle's wing return, an extension of the adaptive windows
(not in the paper): per cell, the Lorentz mass of the points the windows
drop, priced by the midpoint rule (a difference of arctangents per dropped
range) and spread over the band.  Each pin checks it against something other
than its own code: nothing dropped at a vanishing tolerance; a line centred
on a grid point, whose two dropped wings have a closed form; the exact
dropped mass, from the plain and the adaptive sums, within the midpoint
rule's error; the band integral of the plain sum; nesting in the tolerance."""
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from paper_cs_0703028_amd import inputs as I

KB = 1.380649e-23                               # J/K (SI 2019, exact)
ATM = 101325.0


def test_vanishing_tolerance_returns_nothing():
    w = I.small_ragged()
    cells = [0, 7, 8, 100, 209]
    assert (O.wing_return(w.grid, w.lines, 1e-300, cells) == 0).all()
    assert np.array_equal(O.kappa_adaptive(w.grid, w.lines, 1e-300, cells, wings=True),
                          O.kappa(w.grid, w.lines, cells))


@pytest.mark.parametrize("eps", [0.04, 0.1, 0.3])
def test_line_on_a_grid_point_closed_form(eps):
    # dnu = 2^-7 and nu0 integral make r = (nu - nu0)/dnu = 2000 exact; with
    # T = T_ref and no energies the strength ratio is 1 and g = gamma p
    dnu, K = 2.0 ** -7, 640
    base = I.small_ragged().lines
    L = replace(base, nu=np.array([1000.0 + 2000 * dnu]), S=np.array([3e-21]),
                gamma=np.array([0.06]), n_T=np.array([0.7]), E_lower=None, nu0=1000.0,
                dnu=dnu, n_nu=4000, cutoff=K * dnu)
    T, x, p = L.T_ref, 0.2, 1.3
    g = I.linear_T_grid(1, 0.1, ny=1, nz=1)
    g.T, g.x, g.p = np.array([T]), np.array([x]), np.array([p])
    gam = 0.06 * p
    # the adaptive rule for one line: sbar = S / (n_nu dnu), kept while
    # |j - r| dnu <= sqrt(S g / (pi eps sbar) - g^2)
    hw = np.sqrt(gam * L.n_nu * dnu / (np.pi * eps) - gam * gam) / dnu
    kept = int(np.floor(hw))
    assert 0 < kept < K
    u = x * p * ATM / (KB * T) * 1e-6
    both_wings = 2 * (np.arctan((K + 0.5) * dnu / gam) - np.arctan((kept + 0.5) * dnu / gam))
    want = u * 3e-21 * both_wings / (np.pi * dnu * L.n_nu)
    got = O.wing_return(g, L, eps)[0]
    assert got == pytest.approx(want, rel=1e-12)
    # and the midpoint rule against the dropped points summed one by one:
    # relative error below 1/(4 t^2) for points t grid units from the centre
    t = np.arange(kept + 1, K + 1, dtype=np.float64)
    dropped = 2 * (u * 3e-21 * gam / (np.pi * ((t * dnu) ** 2 + gam * gam))).sum() / L.n_nu
    assert abs(got / dropped - 1) <= 1 / (4 * (kept + 1) ** 2)


@pytest.mark.parametrize("wl", ["small_ragged", "plain_8cube"])
@pytest.mark.parametrize("eps", [1e-2, 1e-3, 1e-5])
def test_dropped_mass_and_band_integral(wl, eps):
    w = getattr(I, wl)()
    g, L = w.grid, w.lines
    kp = O.kappa(g, L)
    ka = O.kappa_adaptive(g, L, eps)
    kw = O.kappa_adaptive(g, L, eps, wings=True)
    C = O.wing_return(g, L, eps)
    # the rows carry the constant at every point
    assert np.allclose(kw - ka, C[:, None], rtol=1e-9, atol=0)
    # the exact dropped mass per cell, from the plain and adaptive sums
    D = (kp.sum(1) - ka.sum(1)) / L.n_nu
    assert (D > 0).all()
    rel = np.abs(C / D - 1)
    # the dropped points lie ten and more grid points from their line's
    # centre here (half widths of 5-8 points), where the midpoint rule is
    # within 1/(4 t^2) ~ 2.5e-3; a missing half point at a range end, a
    # factor or a wing would be off by percents
    assert rel.max() <= 1e-3
    # so the band integral of the plain sum is kept to that fraction of what
    # the windows drop
    err_drop = np.abs(ka.mean(1) / kp.mean(1) - 1).max()
    err_wing = np.abs(kw.mean(1) / kp.mean(1) - 1).max()
    print(f"{wl} eps {eps:g}: band mean error {err_drop:.2e} -> {err_wing:.2e}; "
          f"dropped mass rel err {rel.max():.2e}")
    assert err_wing <= 1e-3 * err_drop


def test_nesting_in_the_tolerance():
    # the kept sets nest, so the dropped ranges grow with eps and every
    # range's arctangent mass is positive
    w = I.plain_8cube()
    cells = np.arange(0, w.grid.n_cells, 37, dtype=np.int32)
    prev = np.zeros(len(cells))
    for eps in (1e-6, 1e-5, 1e-4, 1e-3, 1e-2):
        C = O.wing_return(w.grid, w.lines, eps, cells)
        assert (C >= prev).all()
        prev = C
    assert (prev > 0).all()
