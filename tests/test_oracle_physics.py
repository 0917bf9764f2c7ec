"""Pins of the oracle's physics: Eqs. (1), (2) and (4) of Section 3 and the
ideal-gas density, each against something other than the oracle itself.

* Lorentz line sum, Eq. (2): a single line sampled on the uniform grid with a
  window of K points each side equals the Poisson-summation closed form of the
  untruncated comb minus its two tails written with the digamma function:
      sum_{k=-inf}^{inf} 1/((k-phi)^2 + a^2) = (pi/a) sinh(2 pi a)/(cosh(2 pi a) - cos(2 pi phi))
      sum_{k>=0} 1/((k+b)^2 + a^2)          = Im psi(b + i a) / a
  so an off-by-one in the inclusive window, a wrong Delta-nu scale or a
  dropped 1/pi all fail.  With a wide window the sum tends to the normalised
  line integral (2/pi) atan(cutoff/gamma).
* Strength ratio, Eq. (1): special cases where single factors survive.
* Half width: reference point and exact power-law points.
* Density: Loschmidt's constant (CODATA) rescaled to 296 K.
* Planck, Eq. (4): Stefan-Boltzmann (CODATA sigma), Wien's displacement
  constant for the wavenumber peak, Wien and Rayleigh-Jeans limits.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import oracle as O
from paper_cs_0703028_amd import inputs as I

LOSCHMIDT = 2.686780111e25       # m^-3 at 273.15 K, 101.325 kPa (CODATA 2018)
SIGMA = 5.670374419e-8           # W m^-2 K^-4 (CODATA 2018)
WIEN_WAVENUMBER = 1.960998       # cm^-1 / K: peak of B per unit wavenumber


def _one_line_workload(phi, m, gamma, K, dnu=0.01, n_nu=None):
    n_nu = n_nu or (m + K + 40)
    nu0 = 1000.0
    nu_line = nu0 + (m + phi) * dnu
    L = I.Lines(nu=np.array([nu_line]), S=np.array([1e-20]), gamma=np.array([gamma]),
                n_T=np.array([0.5]), E_lower=np.array([800.0]), T_ref=296.0,
                cutoff=K * dnu, nu0=nu0, dnu=dnu, n_nu=n_nu)
    g = I.Grid(1, 1, 1, 0.1, np.array([296.0]), np.array([0.2]), np.array([1.0]))
    return g, L


def _comb_window(a, phi, K):
    """sum over integers k with |k - phi| <= K of 1/((k - phi)^2 + a^2),
    phi in [0,1), as the full comb minus its two tails (exact closed form)."""
    full = math.pi / a * math.sinh(2 * math.pi * a) / (math.cosh(2 * math.pi * a) - math.cos(2 * math.pi * phi))
    # upper tail k >= K+1: b = K+1-phi.  lower tail k <= -K-1 when phi = 0
    # (b = K+1), k <= -K when phi > 0 (the point at -K lies just outside).
    b_lo = K + 1.0 if phi == 0.0 else K + phi
    tail = (special.psi(complex(K + 1 - phi, a)).imag + special.psi(complex(b_lo, a)).imag) / a
    return full - tail


@pytest.mark.parametrize("phi", [0.0, 0.25, 0.5, 0.731, 0.999])
@pytest.mark.parametrize("gamma,K", [(0.05, 500), (0.1, 37), (0.013, 5)])
def test_lorentz_window_sum_poisson_digamma(phi, gamma, K):
    dnu = 0.01
    m = K + 15
    g, L = _one_line_workload(phi, m, gamma, K, dnu)
    r = (L.nu[0] - L.nu0) / dnu
    phi_eff = r - math.floor(r)  # the phase the oracle sees after rounding nu
    kap = O.kappa(g, L)[0]
    u = O.density(296.0, 0.2, 1.0)
    total = kap.sum() * dnu / (u * L.S[0])
    a = gamma / dnu
    exact = a / math.pi * _comb_window(a, phi_eff, K)
    assert abs(total - exact) <= 1e-11 * exact
    # the window is exactly the 2K+1 (or 2K when the centre is off-grid) points
    nz = np.nonzero(kap)[0]
    m_i = math.floor(r)
    assert nz.min() == m_i - K + (1 if phi_eff > 0 else 0) and nz.max() == m_i + K


def test_lorentz_line_integrates_to_strength():
    # a wide window: sum kappa dnu / u -> S (2/pi) atan(cutoff/gamma)
    gamma, K, dnu = 0.07, 4000, 0.01
    g, L = _one_line_workload(0.37, K + 5, gamma, K, dnu)
    kap = O.kappa(g, L)[0]
    u = O.density(296.0, 0.2, 1.0)
    total = kap.sum() * dnu / u
    expect = L.S[0] * 2 / math.pi * math.atan(K * dnu / gamma)
    # rectangle rule on a grid fine against gamma: error << 1e-6
    assert abs(total - expect) <= 2e-6 * expect
    assert abs(total - L.S[0]) <= 2 * gamma / (math.pi * K * dnu) * L.S[0]


def test_lines_outside_grid_contribute_in_grid_part():
    dnu, K = 0.01, 100
    g, L = _one_line_workload(0.5, -30, 0.05, K, dnu, n_nu=200)
    kap = O.kappa(g, L)[0]
    nz = np.nonzero(kap)[0]
    assert nz.min() == 0 and nz.max() == -30 + K


def test_strength_ratio_special_cases():
    c2 = O.c2()
    # T = T_ref: every factor is 1
    assert O.strength_ratio(296.0, 296.0, 1050.0, 1234.0) == pytest.approx(1.0, abs=1e-15)
    # no energies given: ratio 1 at any T
    assert O.strength_ratio(1500.0, 296.0, 1050.0, 0.0, have_E=False) == 1.0
    # E = 0, nu large: only the partition ratio survives, (T_ref/T)^1.5
    assert O.strength_ratio(4 * 296.0, 296.0, 1e6, 0.0) == pytest.approx(0.125, rel=1e-14)
    # hot line: the Boltzmann factor exp(c2 E (1/T_ref - 1/T)) = 8 cancels the
    # partition ratio at T = 4 T_ref
    E = math.log(8.0) / (c2 * (1 / 296.0 - 1 / (4 * 296.0)))
    assert O.strength_ratio(4 * 296.0, 296.0, 1e6, E) == pytest.approx(1.0, rel=1e-13)
    # hot lines grow and cold lines shrink with temperature
    assert O.strength_ratio(1500.0, 296.0, 1e6, 3000.0) > 1.0
    assert O.strength_ratio(1500.0, 296.0, 1e6, 0.0) < 1.0
    # E = 0: the stimulated-emission factor (1-exp(-c2 nu/T))/(1-exp(-c2 nu/T_ref))
    # in the limit nu -> 0 tends to T_ref/T; with the partition ratio: (T_ref/T)^2.5
    assert O.strength_ratio(2 * 296.0, 296.0, 1e-7, 0.0) == pytest.approx(2 ** -2.5, rel=1e-8)


def test_half_width_scaling():
    assert O.half_width(0.07, 0.5, 296.0, 296.0, 1.0) == pytest.approx(0.07, rel=1e-15)
    assert O.half_width(0.07, 0.5, 4 * 296.0, 296.0, 1.0) == pytest.approx(0.035, rel=1e-15)
    assert O.half_width(0.07, 0.75, 296.0 / 16, 296.0, 2.0) == pytest.approx(0.07 * 2 * 8, rel=1e-14)


def test_density_loschmidt():
    n_cm3 = LOSCHMIDT * 273.15 / 296.0 * 1e-6
    assert O.density(296.0, 1.0, 1.0) == pytest.approx(n_cm3, rel=1e-9)
    assert O.density(600.0, 0.25, 2.0) == pytest.approx(n_cm3 * 296 / 600 * 0.5, rel=1e-9)


@pytest.mark.parametrize("T", [300.0, 1000.0, 1800.0])
def test_planck_stefan_boltzmann(T):
    # pi * integral of B over wavenumber = sigma T^4  (B per cm^-1, W m^-2 sr^-1)
    f = lambda nu: O.planck(nu, T)
    peak = WIEN_WAVENUMBER * T
    val = sum(integrate.quad(f, lo, hi, epsabs=0, epsrel=1e-13, limit=400)[0]
              for lo, hi in ((1e-12, peak), (peak, 10 * peak), (10 * peak, 60 * peak)))
    assert math.pi * val == pytest.approx(SIGMA * T ** 4, rel=1e-9)


def test_planck_peak_and_limits():
    T = 1234.0
    nus = np.linspace(0.5 * WIEN_WAVENUMBER * T, 1.5 * WIEN_WAVENUMBER * T, 200001)
    vals = np.array([O.planck(v, T) for v in nus])
    assert nus[vals.argmax()] == pytest.approx(WIEN_WAVENUMBER * T, rel=2e-6)
    c1, c2 = O.c1(), O.c2()
    # Wien: x = c2 nu / T >> 1
    nu = 60 * T / c2
    assert O.planck(nu, T) == pytest.approx(c1 * nu ** 3 * math.exp(-c2 * nu / T), rel=1e-25 + 1e-26 + 1e-12)
    # Rayleigh-Jeans: x << 1 -> B = c1 nu^2 T / c2 (1 - x/2 + x^2/12)
    nu = 1e-4 * T / c2
    x = c2 * nu / T
    assert O.planck(nu, T) == pytest.approx(c1 * nu ** 2 * T / c2 * (1 - x / 2 + x * x / 12), rel=1e-12)
    # cold wall
    assert O.planck(1000.0, 0.0) == 0.0
    # the constants themselves: c2 = h c / k in cm K, c1 = 2 h c^2 1e8
    assert c2 == pytest.approx(1.438776877, rel=1e-9)
    assert c1 == pytest.approx(1.191042972e-8, rel=1e-9)
