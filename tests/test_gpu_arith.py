"""FP32 arithmetic of gfx950 against exact references (the paper's Section 2
experiments, Table 2), through rt_arith_eval.

Bars: add, sub, mul, fma, the unfused multiply-add, the fma error term, the
composites and the compiler's division are IEEE 754 binary32, round to
nearest even, gradual underflow -- bit for bit.  v_exp_f32, v_log_f32,
v_rcp_f32, v_rsq_f32 and v_sqrt_f32 are within 1 ulp (their documented
accuracy) over normal inputs and results.  The largest errors seen are
printed for the record.
"""
import numpy as np
import pytest

from oracle import arith as A

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_cs_0703028_amd import rtlbl
    t = rtlbl.Tracer(0)

    def run(op, *xs):
        ts = [torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda() for x in xs]
        out = t.arith_eval(op, *ts)
        torch.cuda.synchronize()
        return out.cpu().numpy()
    yield run
    t.close()


def bits(x):
    return np.asarray(x, np.float32).view(np.uint32)


def same(got, want):
    g, w = bits(got), bits(want)
    bad = np.nonzero(g != w)[0]
    assert bad.size == 0, f"{bad.size} mismatches, first at {bad[:5]}: {g[bad[:5]]} vs {w[bad[:5]]}"


def wide(rng, n, lo=-60, hi=60):
    """Random binary32 with log-uniform magnitudes and random signs."""
    m = rng.uniform(1, 2, n)
    s = rng.choice([-1.0, 1.0], n)
    return (s * np.ldexp(m, rng.integers(lo, hi, n))).astype(np.float32)


def test_add_sub_mul_div_correctly_rounded(ev):
    rng = np.random.default_rng(1)
    n = 1 << 20
    for x, y in [(rng.uniform(1, 2, n), rng.uniform(1, 2, n)),
                 (wide(rng, n), wide(rng, n)),
                 (wide(rng, n, -140, -100), wide(rng, n, -30, 0))]:   # subnormal results
        x = x.astype(np.float32); y = y.astype(np.float32)
        same(ev("add", x, y), A.ref_add(x, y))
        same(ev("sub", x, y), A.ref_sub(x, y))
        same(ev("mul", x, y), A.ref_mul(x, y))
    x, y = wide(rng, n, -60, 60), wide(rng, n, -60, 60)
    same(ev("div", x, y), A.ref_div(x, y))


def test_fma_is_fused_and_mul_add_is_not(ev):
    rng = np.random.default_rng(2)
    n = 1 << 15
    x = rng.uniform(1, 2, n).astype(np.float32)
    y = rng.uniform(1, 2, n).astype(np.float32)
    z = -rng.uniform(1, 4, n).astype(np.float32)
    same(ev("fma", x, y, z), A.ref_fma(x, y, z))
    same(ev("mul_add", x, y, z), A.ref_mul_add(x, y, z))
    # the paper's MAD(x, y, -x*y): 0 for an unfused unit; here the exact
    # rounding error of the product, non-zero for most inputs
    err = ev("fma_err", x, y)
    same(err, A.ref_fma_err(x, y))
    print(f"fma(x, y, -x*y) non-zero for {np.mean(err != 0):.3f} of U[1,2)^2")
    assert np.mean(err != 0) > 0.5


def test_table2_ties_and_overflow(ev):
    i = np.arange(1, 41)
    p = np.ldexp(1.0, -i).astype(np.float32)
    got = ev("sub", np.full(40, 1.5, np.float32), p)
    same(got, [A.table2_tie(k) for k in i])
    got = ev("add_sub", np.ones(40, np.float32), np.full(40, 0.5, np.float32), p)
    same(got, [A.table2_tie(k) for k in i])
    got = ev("sub_sub", np.full(40, 1.5, np.float32), p, np.full(40, 1.5, np.float32))
    same(got, [A.table2_tie_back(k) for k in i])
    M = np.finfo(np.float32).max
    got = ev("add_sub", np.full(1, M, np.float32), np.full(1, M, np.float32), np.full(1, M, np.float32))
    assert np.isposinf(got[0]) and np.isposinf(A.table2_overflow())


def test_product_symmetry_scaling_and_error(ev):
    rng = np.random.default_rng(4)
    n = 1 << 23
    x = rng.uniform(1, 2, n).astype(np.float32)
    y = rng.uniform(1, 2, n).astype(np.float32)
    p = ev("mul", x, y)
    same(ev("mul", -x, y), -p)
    same(ev("mul", x, -y), -p)
    same(ev("mul", -x, -y), p)
    same(ev("mul", (2 * x).astype(np.float32), y), (2 * p).astype(np.float32))
    # error of the product in ulps over the paper's two regions (y below and
    # above 2/x); round to nearest: within [-1/2, 1/2]
    e = A.ulp_error(p, x.astype(np.float64) * y.astype(np.float64))
    lo = y < 2 / x
    for name, sel in (("y < 2/x", lo), ("y >= 2/x", ~lo)):
        print(f"x*y - exact, {name}: [{e[sel].min():.5f}, {e[sel].max():.5f}] ulp")
    assert np.abs(e).max() <= 0.5
    same(p, A.ref_mul(x, y))


def test_products_near_one_exhaustive(ev):
    # (1 + 2^-23)(1 + 2^-23 i), every i < 2^23
    i = np.arange(1 << 23, dtype=np.float64)
    a = np.full(i.size, 1 + 2.0 ** -23, np.float32)
    b = (1 + i * 2.0 ** -23).astype(np.float32)
    same(ev("mul", a, b), A.ref_mul(a, b))


def test_subnormals_and_nans(ev):
    sub = np.ldexp(1.0, -np.arange(127, 150)).astype(np.float32)       # 2^-127 .. 2^-149
    sub = np.concatenate([sub, -sub, (sub * 3).astype(np.float32)])
    same(ev("copy", sub), sub)
    same(ev("add", sub, np.zeros_like(sub)), sub)
    same(ev("mul", sub, np.ones_like(sub)), sub)
    # NaN payloads through a copy and through an operation
    nan_bits = np.array([0x7FC00001, 0x7F800001, 0xFFA00000], np.uint32)   # quiet, signalling, signalling
    nans = nan_bits.view(np.float32)
    c = ev("copy", nans)
    assert np.all(np.isnan(c))
    s = ev("add", nans, np.zeros_like(nans))
    assert np.all(np.isnan(s))
    quiet = (bits(s) & 0x00400000) != 0
    print(f"copy keeps NaN bits: {bool(np.all(bits(c) == nan_bits))}; "
          f"add returns quiet NaNs: {bool(np.all(quiet))}")


def _ulps(got, exact):
    return np.abs(A.ulp_error(got, exact))


def test_hardware_transcendentals_within_one_ulp(ev):
    rng = np.random.default_rng(5)
    n = 1 << 22
    cases = {
        "exp2": (rng.uniform(-125.0, 127.9, n).astype(np.float32), A.ref_exp2),
        "log2": (np.ldexp(rng.uniform(1, 2, n), rng.integers(-125, 127, n)).astype(np.float32), A.ref_log2),
        "rcp": (np.ldexp(rng.uniform(1, 2, n), rng.integers(-125, 125, n)).astype(np.float32), A.ref_rcp),
        "rsq": (np.ldexp(rng.uniform(1, 2, n), rng.integers(-125, 127, n)).astype(np.float32), A.ref_rsq),
        "sqrt": (np.ldexp(rng.uniform(1, 2, n), rng.integers(-125, 127, n)).astype(np.float32), A.ref_sqrt64),
    }
    # dense near the points the march and line sum use: 2^x for x in [-1, 0]
    # (transmittances), 1/x in [1, 2)
    cases["exp2_unit"] = (rng.uniform(-1.0, 0.0, n).astype(np.float32), A.ref_exp2)
    cases["rcp_unit"] = (rng.uniform(1.0, 2.0, n).astype(np.float32), A.ref_rcp)
    worst = {}
    for name, (x, ref) in cases.items():
        op = name.split("_")[0]
        e = _ulps(ev(op, x), ref(x))
        worst[name] = float(e.max())
        print(f"{name}: max {e.max():.4f} ulp, mean {e.mean():.4f}")
    assert all(v <= 1.0 for v in worst.values()), worst
