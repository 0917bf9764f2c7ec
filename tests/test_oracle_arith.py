"""Pins of the exact references of the FP32 arithmetic characterisation
(oracle/arith.py), each against something other than itself: hand-worked
IEEE 754 cases, numpy's own binary64 -> binary32 conversion, 50-digit
mpmath values, and an independent long-double evaluation."""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle import arith as A

F = Fraction


def bits(x):
    return np.asarray(x, np.float32).view(np.uint32)


@pytest.mark.parametrize("q, want", [
    (F(1) + F(1, 2 ** 24), 1.0),                       # tie -> even (1.0)
    (F(1) + F(3, 2 ** 24), 1.0 + 2.0 ** -22),          # tie -> even (...10)
    (F(1) + F(1, 2 ** 23) + F(1, 2 ** 25), 1.0 + 2.0 ** -23),  # below the tie
    (F(3, 2) - F(1, 2 ** 24), 1.5),                    # the paper's i = 24
    (F(3, 2) - F(1, 2 ** 23), 1.5 - 2.0 ** -23),
    (F(1, 2 ** 150), 0.0),                             # half the smallest subnormal -> 0 (even)
    (F(3, 2 ** 150), 2.0 ** -148),                     # 1.5 subnormal ulps -> 2 (even)
    (F(5, 2 ** 151), 2.0 ** -149),                     # 1.25 ulps -> 1
    (F(-7, 2 ** 3), -0.875),
])
def test_round_fraction_known_cases(q, want):
    assert bits(A.round_fraction_f32(q)) == bits(np.float32(want))


def test_round_fraction_overflow_threshold():
    top = F(2 ** 24 - 1) * F(2) ** 104                 # largest finite binary32
    half = F(2) ** 103                                 # half an ulp there
    assert A.round_fraction_f32(top + half - F(1, 2 ** 60)) == np.float32(top)
    assert np.isposinf(A.round_fraction_f32(top + half))   # tie -> even neighbour 2^128
    assert np.isneginf(A.round_fraction_f32(-(top + 2 * half)))


def test_round_fraction_matches_numpy_conversion():
    # numpy rounds binary64 to binary32 with the same rule; binary64 values
    # are exact fractions, so both must agree bit for bit
    rng = np.random.default_rng(7)
    v = np.concatenate([
        rng.uniform(-4, 4, 3000),
        np.ldexp(rng.uniform(1, 2, 2000), rng.integers(-160, 128, 2000)),
        # exact ties of binary32 (25 significant bits, last one set)
        np.ldexp((rng.integers(2 ** 24, 2 ** 25, 1000) | 1).astype(np.float64), rng.integers(-170, 90, 1000)),
    ])
    for x in v:
        assert bits(A.round_fraction_f32(F(float(x)))) == bits(np.float32(x)), x


def test_ulp32_known_values():
    got = A.ulp32([1.0, 1.5, 2.0, 3.99, 2.0 ** -126, 2.0 ** -130, 2.0 ** 127])
    want = [2.0 ** -23, 2.0 ** -23, 2.0 ** -22, 2.0 ** -22, 2.0 ** -149, 2.0 ** -149, 2.0 ** 104]
    assert np.array_equal(got, want)
    assert A.ulp_error(np.float32(1.0 + 2.0 ** -23), 1.0) == pytest.approx(1.0)


def _cases(rng, n):
    a = np.ldexp(rng.uniform(1, 2, n), rng.integers(-20, 20, n)).astype(np.float32)
    b = np.ldexp(rng.uniform(1, 2, n), rng.integers(-20, 20, n)).astype(np.float32)
    s = rng.choice([-1, 1], n).astype(np.float32)
    return a, b * s


def test_double_rounding_is_innocuous_for_basic_ops():
    # the binary64 route of ref_add/sub/mul/div/sqrt against exact fractions
    rng = np.random.default_rng(11)
    a, b = _cases(rng, 4000)
    # near-ties of the product: significands whose exact product has a
    # 25th bit of one followed by few ones
    m = (rng.integers(2 ** 22, 2 ** 23, 500) * 2 + 1).astype(np.float32) / np.float32(2 ** 23)
    a = np.concatenate([a, m]); b = np.concatenate([b, (m[::-1] + np.float32(0.5)).astype(np.float32)])
    for x, y in zip(a, b):
        fx, fy = F(float(x)), F(float(y))
        assert bits(A.ref_add(x, y)) == bits(A.round_fraction_f32(fx + fy))
        assert bits(A.ref_sub(x, y)) == bits(A.round_fraction_f32(fx - fy))
        assert bits(A.ref_mul(x, y)) == bits(A.round_fraction_f32(fx * fy))
        assert bits(A.ref_div(x, y)) == bits(A.round_fraction_f32(fx / fy))
    # sqrt: round(sqrt(q)) from the exact square root's bracketing
    for x in np.abs(a[:2000]):
        r = A.ref_sqrt(x)
        fr, fx = F(float(r)), F(float(x))
        up = F(float(np.nextafter(r, np.float32(np.inf))))
        dn = F(float(np.nextafter(r, np.float32(0))))
        # r is the nearest: (r - half ulp)^2 <= x <= (r + half ulp)^2
        assert ((fr + dn) / 2) ** 2 <= fx <= ((fr + up) / 2) ** 2


def test_fma_reference_against_long_double():
    # for operands in [1, 2) the long-double x*y + z is exact (48 + 24 bits
    # within a 64-bit significand), so one rounding of it is the fma
    rng = np.random.default_rng(3)
    x = rng.uniform(1, 2, 3000).astype(np.float32)
    y = rng.uniform(1, 2, 3000).astype(np.float32)
    z = -rng.uniform(1, 4, 3000).astype(np.float32)
    ld = np.longdouble
    exact = x.astype(ld) * y.astype(ld) + z.astype(ld)
    want = np.array([A.round_fraction_f32(F(int(e * ld(2) ** 70), 2 ** 70)) for e in exact], np.float32)
    assert np.array_equal(bits(A.ref_fma(x, y, z)), bits(want))
    # and fma(x, y, -round(x y)) is the product's rounding error
    err = A.ref_fma_err(x, y)
    p = A.ref_mul(x, y).astype(ld)
    assert np.array_equal(err.astype(ld), x.astype(ld) * y.astype(ld) - p)


def test_transcendental_references_against_mpmath():
    mpmath.mp.dps = 50
    xs = np.array([-126.0, -3.3, -0.001, 0.0, 0.5, 1.0, 7.25, 127.9], np.float32)
    for x in xs:
        e = mpmath.power(2, mpmath.mpf(float(x)))
        assert abs(A.ref_exp2(x) - float(e)) <= 1e-15 * float(e)
    for x in np.array([1e-30, 0.1, 1.0, 1.5, 3.0, 1e30], np.float32):
        X = mpmath.mpf(float(x))
        assert abs(A.ref_log2(x) - float(mpmath.log(X, 2))) <= 1e-15 * max(1.0, abs(float(mpmath.log(X, 2))))
        assert abs(A.ref_rcp(x) - float(1 / X)) <= 1e-15 * float(1 / X)
        assert abs(A.ref_rsq(x) - float(1 / mpmath.sqrt(X))) <= 1e-15 * float(1 / mpmath.sqrt(X))


def test_table2_vectors_under_ieee():
    # hand-worked: 1.5 - 2^-i is exact up to i = 23; i = 24 is a tie that
    # goes to the even neighbour 1.5; beyond, 1.5
    for i in range(1, 24):
        assert A.table2_tie(i) == np.float32(1.5 - 2.0 ** -i)
        assert A.table2_tie_back(i) == np.float32(-(2.0 ** -i))
    for i in (24, 25, 30, 40):
        assert A.table2_tie(i) == np.float32(1.5)
        assert A.table2_tie_back(i) == 0
    assert np.isposinf(A.table2_overflow())
