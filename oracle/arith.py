"""Exact references for the FP32 arithmetic characterisation of the device
(the paper's Section 2: test vectors of Table 2 and the observations around
it on rounding, multiply-add, products, subnormals and NaNs).

Test infrastructure only: the test-suite may import this module; the library
product never does.

"Correct" is IEEE 754 binary32 with rounding to nearest, ties to even, and
gradual underflow:
- round_fraction_f32 rounds an exact rational once, by that rule, written out
  from the definition (binade, ulp, remainder against one half);
- x + y, x - y, x * y, x / y and sqrt(x) of binary32 operands: the binary64
  result rounded again to binary32.  For these five operations binary64
  carries at least 2*24 + 2 bits, which makes the second rounding innocuous
  (Figueroa, "When is double rounding innocuous?", 1995); the tests check
  this against round_fraction_f32 on random and near-tie inputs;
- fma(x, y, z): the exact x*y + z as a fraction, rounded once;
- 2^x, log2 x, 1/x, 1/sqrt x: binary64 values, within ~1e-16 relative of
  the exact ones, enough to measure binary32 errors to ~1e-8 ulp.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

F32_MAX = Fraction(2 ** 24 - 1) * Fraction(2) ** (127 - 23)
_EMIN = -126          # smallest normal exponent
_P = 24               # binary32 significand bits


def round_fraction_f32(q: Fraction) -> np.float32:
    """The binary32 value nearest to q (ties to even), with gradual underflow
    and overflow to infinity.  A zero q gives +0."""
    if q == 0:
        return np.float32(0.0)
    sign = -1 if q < 0 else 1
    a = -q if q < 0 else q
    # binade: 2^e <= a < 2^(e+1)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    u = max(e, _EMIN) - (_P - 1)          # exponent of the ulp at a
    m = a / Fraction(2) ** u              # a in ulps
    n = m.numerator // m.denominator
    r = m - n
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and n % 2 == 1):
        n += 1
    v = Fraction(n) * Fraction(2) ** u
    # the overflow threshold is halfway between F32_MAX and 2^128: a value
    # there rounds to the even neighbour 2^128, i.e. to infinity
    if v > F32_MAX:
        return np.float32(sign * np.inf)
    return np.float32(sign * float(v))    # v is exact in binary64


def f32_fraction(x) -> Fraction:
    """Exact value of a finite binary32 (or binary64) number."""
    return Fraction(float(x))


def ulp32(v) -> np.ndarray:
    """Spacing of binary32 numbers at |v| (|v| a real number given in
    binary64): 2^(floor(log2 |v|) - 23) for normal magnitudes, 2^-149 below."""
    v = np.abs(np.asarray(v, np.float64))
    m, e = np.frexp(v)                    # v = m 2^e, m in [0.5, 1)
    u = np.ldexp(1.0, e - 24)
    return np.where(v < 2.0 ** _EMIN, 2.0 ** -149, u)


def ulp_error(got, exact) -> np.ndarray:
    """(got - exact) in ulps of binary32 at the exact value."""
    got = np.asarray(got, np.float32).astype(np.float64)
    exact = np.asarray(exact, np.float64)
    return (got - exact) / ulp32(exact)


# ------------------------------------------------ correctly rounded results
def _f64(x):
    return np.asarray(x, np.float32).astype(np.float64)


def ref_add(x, y):
    return (_f64(x) + _f64(y)).astype(np.float32)


def ref_sub(x, y):
    return (_f64(x) - _f64(y)).astype(np.float32)


def ref_mul(x, y):
    return (_f64(x) * _f64(y)).astype(np.float32)


def ref_div(x, y):
    return (_f64(x) / _f64(y)).astype(np.float32)


def ref_sqrt(x):
    return np.sqrt(_f64(x)).astype(np.float32)


def ref_fma(x, y, z) -> np.ndarray:
    """fma(x, y, z) rounded once, element by element through fractions."""
    x, y, z = (np.asarray(t, np.float32).ravel() for t in (x, y, z))
    out = np.empty(x.size, np.float32)
    for k in range(x.size):
        out[k] = round_fraction_f32(f32_fraction(x[k]) * f32_fraction(y[k]) + f32_fraction(z[k]))
    return out


def ref_mul_add(x, y, z):
    """x * y rounded, then + z rounded: the unfused multiply-add."""
    return ref_add(ref_mul(x, y), z)


def ref_fma_err(x, y) -> np.ndarray:
    """x*y - round(x*y): exact, and representable in binary32 unless the
    product underflows, computed from fractions."""
    x, y = (np.asarray(t, np.float32).ravel() for t in (x, y))
    p = ref_mul(x, y)
    out = np.empty(x.size, np.float32)
    for k in range(x.size):
        out[k] = round_fraction_f32(f32_fraction(x[k]) * f32_fraction(y[k]) - f32_fraction(p[k]))
    return out


# ------------------------------------------ binary64 references, for ulps
def ref_exp2(x):
    return np.exp2(_f64(x))


def ref_log2(x):
    return np.log2(_f64(x))


def ref_rcp(x):
    return 1.0 / _f64(x)


def ref_rsq(x):
    return 1.0 / np.sqrt(_f64(x))


def ref_sqrt64(x):
    return np.sqrt(_f64(x))


# --------------------------------------------------- the Table 2 vectors
def table2_tie(i: int) -> np.float32:
    """1.5 - 2^-i, rounded once."""
    return round_fraction_f32(Fraction(3, 2) - Fraction(1, 2 ** int(i)))


def table2_tie_back(i: int) -> np.float32:
    """(1.5 - 2^-i) - 1.5 with the inner difference rounded."""
    return round_fraction_f32(f32_fraction(table2_tie(i)) - Fraction(3, 2))


def table2_overflow() -> np.float32:
    """(M + M) - M for the largest finite M: M + M overflows."""
    m = f32_fraction(np.float32(F32_MAX))
    s = round_fraction_f32(m + m)
    if np.isinf(s):
        return s
    return round_fraction_f32(f32_fraction(s) - m)
