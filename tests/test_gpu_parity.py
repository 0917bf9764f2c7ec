"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars (stated per result):
* traversal (integer work): cells, segment counts, origins and directions
  bit-exact; lengths equal to the oracle's FP64 length rounded to FP32;
* kappa and Planck tables: 1e-5 relative per element (the Planck table, all
  FP32, also within its own rounding bound of 1e-6), exact zeros where the
  oracle has zeros (window membership is integer work);
* per-cell absorbed and emitted power and the energy balance: 1e-5 relative
  (the floating-point tolerance of the method's FP32 path); cells the oracle
  leaves at exactly zero must be exactly zero.
"""
import math
from dataclasses import replace

import numpy as np
import pytest

import oracle_pool
from paper_cs_0703028_amd import inputs as I

pytestmark = pytest.mark.gpu

REL = 1e-5
U = 1 << 21


@pytest.fixture(scope="module")
def rt():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_cs_0703028_amd import rtlbl
    return rtlbl


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    return oracle


def _tracer(rt, w):
    t = rt.Tracer(0)
    t.setup_grid(w.grid)
    t.setup_lines(w.lines)
    return t


def _rel(g, o):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    nz = o != 0
    assert (g[~nz] == 0).all(), "GPU nonzero where the oracle is exactly zero"
    return np.abs(g[nz] - o[nz]) / np.abs(o[nz])


def _say(msg):
    print(msg, flush=True)


# ----------------------------------------------------------------- traversal
@pytest.mark.parametrize("wl", ["small_ragged", "plain_8cube", "plain_32cube"])
def test_segments_bit_exact(rt, O, wl):
    w = getattr(I, wl)()
    t = _tracer(rt, w)
    g = w.grid
    rng = np.random.default_rng(5)
    begins = [0, int(rng.integers(0, max(w.n_rays - 600, 1)))]
    for b in begins:
        _say(f"segments {wl} rays [{b}, {b + 600})")
        counts, cells, lens, Og, Dg = t.debug_segments(w.seed, b, 600)
        Oo, Do, _ = O.rays(w.seed, b, 600, g.nx, g.ny, g.nz)
        assert (Og == Oo).all() and (Dg == Do).all()
        for r in range(600):
            c_o, l_o = O.segments(g.nx, g.ny, g.nz, g.cell_m * 100.0, Oo[r], Do[r])
            assert counts[r] == len(c_o)
            assert (cells[r, :counts[r]] == c_o).all()
            np.testing.assert_array_equal(lens[r, :counts[r]], l_o.astype(np.float32))
    t.close()


# ------------------------------------------------------------- kappa, Planck
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("wl", ["small_ragged", "plain_8cube"])
def test_kappa_and_planck_tables(rt, O, wl, mode):
    w = getattr(I, wl)()
    t = _tracer(rt, w)
    _say(f"kappa {wl} mode {mode}")
    kap, B = t.compute_kappa(mode)
    ld = t.required_pitch()
    assert ld % 256 == 0 and ld >= w.lines.n_nu
    kg = kap.cpu().numpy()
    bg = B.cpu().numpy()
    ko = O.kappa(w.grid, w.lines)
    bo = O.planck_rows(w.grid, w.lines)
    assert (kg[:, w.lines.n_nu:] == 0).all() and (bg[:, w.lines.n_nu:] == 0).all()
    rk = _rel(kg[:, :w.lines.n_nu], ko)
    rb = _rel(bg[:, :w.lines.n_nu], bo)
    _say(f"  kappa rel err max {rk.max():.3e} median {np.median(rk):.3e}; planck {rb.max():.3e}")
    assert rk.max() <= REL
    # the table is evaluated in FP32 (pair arguments, Cody-Waite exponential):
    # at most about 14 roundings of 2^-24 each (nu, nu^3 and c1: 8; the
    # exponential and its subtraction of 1, which can amplify by 2.5: 5; the
    # division: 1), i.e. 8.3e-7
    assert rb.max() <= 1e-6
    st = t.stats()
    assert st["line_evals"] > 0
    t.close()


# --------------------------------------------------------------------- march
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("wl,T_wall", [("plain_8cube", 0.0), ("small_ragged", 1250.0)])
def test_tallies_match_oracle(rt, O, wl, T_wall, prec):
    w = getattr(I, wl)()
    w.grid.T_wall = T_wall
    t = _tracer(rt, w)
    mode = 1 if prec == 1 else 0
    _say(f"tallies {wl} T_wall {T_wall} prec {prec}")
    t.compute_kappa(mode)
    t.trace_rays(w.seed, w.n_rays, 0, w.n_rays, prec)
    ag, eg, bg = t.tally()
    res = O.run(w.grid, w.lines, w.n_rays, seed=w.seed)
    ra = _rel(ag, res["absorbed"])
    re = _rel(eg, res["emitted"])
    rbal = np.abs(bg - res["balance"]) / np.maximum(np.abs(res["balance"]), 1e-300)
    _say(f"  absorbed max {ra.max():.3e} median {np.median(ra):.3e}; emitted max {re.max():.3e};"
         f" balance {rbal}")
    assert ra.max() <= REL and re.max() <= REL
    for k in range(4):
        if res["balance"][k] == 0:
            assert bg[k] == 0
        else:
            assert rbal[k] <= REL
    ent, emi, ab, esc = bg
    assert abs(ent + emi - ab - esc) <= 1e-5 * (ent + emi)
    st = t.stats()
    assert st["rays"] == w.n_rays and st["updates"] == st["segments"] * w.lines.n_nu
    t.close()


def test_ray_ranges_add_up(rt, O):
    """Tracing [0, n) in pieces gives the tallies of one call (same rays)."""
    w = I.small_ragged()
    t = _tracer(rt, w)
    t.compute_kappa(0)
    t.trace_rays(w.seed, w.n_rays, 0, w.n_rays)
    a1, e1, b1 = t.tally()
    t.reset_tally()
    for b, c in ((300, 400), (0, 100), (100, 200)):
        t.trace_rays(w.seed, w.n_rays, b, c)
    a2, e2, b2 = t.tally()
    # exact fixed-point sums: the split of the rays over calls does not matter
    assert np.array_equal(a2, a1) and np.array_equal(e2, e1) and np.array_equal(b2, b1)
    t.close()


def test_slab_axis_normal_closed_form(rt, O):
    """1-cell slab, L = 1 m, walls at 1500 K: I_exit = I_w e^{-kL} + B (1 - e^{-kL})."""
    w = I.slab_1cell()
    t = _tracer(rt, w)
    t.compute_kappa(1)
    Os = np.array([[0, U // 2 + 1, U // 2 + 1], [U, 3, U - 5], [7, 0, U // 3 * 2 + 1]], np.int64)
    Ds = np.array([[1 << 20, 0, 0], [-(1 << 20), 0, 0], [0, 1 << 20, 0]], np.int64)
    _say("slab explicit rays")
    ex = t.trace_explicit(Os, Ds, 1.0, prec=1, want_exit=True)
    kap = O.kappa(w.grid, w.lines)[0]
    B = O.planck_rows(w.grid, w.lines)[0]
    nu = w.lines.nu0 + np.arange(w.lines.n_nu) * w.lines.dnu
    Bw = np.array([O.planck(v, 1500.0) for v in nu])
    tr = np.exp(-kap * 100.0)
    expect = Bw * tr + B * (1.0 - tr)
    for r in range(3):
        err = np.abs(ex[r] - expect) / expect
        assert err.max() <= REL
    t.close()


def test_abi_errors(rt):
    w = I.small_ragged()
    t = rt.Tracer(0)
    # call order
    with pytest.raises(rt.RtError) as e:
        t.trace_rays(0, 10)
    assert e.value.status == rt.RT_ESTATE
    t.setup_grid(w.grid)
    # kappa before the line list
    assert t.raw_status("rt_compute_kappa", 0, None, None, 256) == rt.RT_ESTATE
    # invalid values
    bad = I.small_ragged().grid
    bad.T = bad.T.copy()
    bad.T[3] = -1.0
    with pytest.raises(rt.RtError) as e:
        t.setup_grid(bad)
    assert e.value.status == rt.RT_EINVAL and "T" in t.last_error()
    L = I.small_ragged().lines
    L.cutoff = 5.005
    with pytest.raises(rt.RtError) as e:
        t.setup_lines(L)
    assert e.value.status == rt.RT_EINVAL and "integer" in t.last_error()
    t.setup_lines(w.lines)
    kap, B = t.alloc_tables()
    assert t.raw_status("rt_compute_kappa", 0, kap.data_ptr(), B.data_ptr(), 100) == rt.RT_EINVAL
    assert t.raw_status("rt_compute_kappa", 7, kap.data_ptr(), B.data_ptr(), kap.shape[1]) == rt.RT_EINVAL
    t.compute_kappa(0, kap, B)
    assert t.raw_status("rt_trace_rays", 0, 10, 5, 6, 0) == rt.RT_EINVAL
    assert t.raw_status("rt_trace_rays", 0, 0, 0, 0, 0) == rt.RT_EINVAL
    assert t.raw_status("rt_trace_rays", 0, 10, 0, 5, 3) == rt.RT_EINVAL
    # a ray that does not start on the boundary
    with pytest.raises(rt.RtError):
        t.trace_explicit(np.array([[5, 5, 5]]), np.array([[1, 0, 0]]), 1.0)
    t.close()


# ------------------------------------------------------------- full size
@pytest.mark.slow
def test_full_size_32cube_sampled(rt, O):
    """The 32^3 / 20,000-line / 50,000-point workload at full size on the GPU:
    kappa of 64 sampled cells (every point) and the tallies of a sampled ray
    range against the oracle (which computes only the cells those rays
    visit)."""
    w = I.plain_32cube()
    t = _tracer(rt, w)
    _say("full-size 32^3 compute_kappa (plain)")
    kap, B = t.compute_kappa(0)
    rng = np.random.default_rng(11)
    cells = np.sort(rng.choice(w.grid.n_cells, 64, replace=False)).astype(np.int32)
    kg = kap[cells.tolist()].cpu().numpy()[:, :w.lines.n_nu]
    ko = O.kappa(w.grid, w.lines, cells)
    rk = _rel(kg, ko)
    _say(f"  kappa sampled max rel {rk.max():.3e}")
    assert rk.max() <= REL
    begin, count = 777_000, 6
    _say(f"full-size 32^3 trace rays [{begin}, {begin + count}) of 2^20")
    t.trace_rays(w.seed, w.n_rays, begin, count, 0)
    ag, eg, bg = t.tally()
    res = O.run(w.grid, w.lines, w.n_rays, seed=w.seed, begin=begin, count=count,
                cells_needed_only=True)
    ra = _rel(ag, res["absorbed"])
    re = _rel(eg, res["emitted"])
    _say(f"  absorbed max rel {ra.max():.3e}, emitted {re.max():.3e}")
    assert ra.max() <= REL and re.max() <= REL
    t.close()


@pytest.mark.slow
def test_full_size_32cube_precision_form_sampled(rt, O):
    """The precision form at the 32^3 workload's full size: the compensated
    line sum and the FP32 Planck table of 64 sampled cells (every point), and
    a ray range traced with the precision march (FP64 tally partials), all
    against the oracle."""
    w = I.plain_32cube()
    t = _tracer(rt, w)
    _say("full-size 32^3 compute_kappa (compensated, with the Planck table)")
    kap, B = t.compute_kappa(rt.KAPPA_COMPENSATED)
    assert B is not None
    rng = np.random.default_rng(12)
    cells = np.sort(rng.choice(w.grid.n_cells, 64, replace=False)).astype(np.int32)
    nz = w.lines.n_nu
    kg = kap[cells.tolist()].cpu().numpy()[:, :nz]
    bg = B[cells.tolist()].cpu().numpy()[:, :nz]
    rk = _rel(kg, O.kappa(w.grid, w.lines, cells))
    rb = _rel(bg, O.planck_rows(w.grid, w.lines, cells))
    _say(f"  kappa sampled max rel {rk.max():.3e}, planck {rb.max():.3e}")
    assert rk.max() <= REL and rb.max() <= 1e-6
    begin, count = 333_333, 6
    _say(f"full-size 32^3 precision march, rays [{begin}, {begin + count}) of 2^20")
    t.trace_rays(w.seed, w.n_rays, begin, count, rt.TALLY_F64)
    ag, eg, bg_ = t.tally()
    res = O.run(w.grid, w.lines, w.n_rays, seed=w.seed, begin=begin, count=count,
                cells_needed_only=True)
    ra, re = _rel(ag, res["absorbed"]), _rel(eg, res["emitted"])
    rbal = _rel(bg_, res["balance"])
    _say(f"  absorbed max rel {ra.max():.3e}, emitted {re.max():.3e}, balance {rbal.max():.3e}")
    assert ra.max() <= REL and re.max() <= REL and rbal.max() <= REL
    t.close()


def _check_tallies(tag, got, ref):
    ag, eg, bg = got
    ra = _rel(ag, ref["absorbed"])
    re_ = _rel(eg, ref["emitted"])
    rb = _rel(bg, ref["balance"])
    _say(f"  {tag}: absorbed max {ra.max():.3e} median {np.median(ra):.3e}, "
         f"emitted max {re_.max():.3e}, balance {rb.max():.3e}")
    assert ra.max() <= REL and re_.max() <= REL and rb.max() <= REL


@pytest.mark.slow
def test_plain_8cube_coherent_call_matches_oracle(rt, O):
    """The 8^3 workload with 2^15 rays in one rt_trace_rays call: a batch of
    2^15 rays or more runs in the coherent order, the path full-size calls
    take.  Per cell against the oracle over the same rays (marched on host
    threads)."""
    w = I.plain_8cube()
    n = 1 << 15
    t = _tracer(rt, w)
    t.compute_kappa(0)
    _say(f"plain_8cube: {n} rays in one call")
    t.trace_rays(w.seed, n, 0, n, rt.TALLY_F32)
    got = t.tally()
    assert t.stats()["march_launches"] == 1
    t.close()
    _say(f"  oracle on {oracle_pool.threads()} threads")
    _check_tallies("8^3, 2^15 rays, coherent order", got,
                   oracle_pool.run(w.grid, w.lines, n, seed=w.seed))


@pytest.mark.slow
def test_32cube_coherent_call_two_chunks_matches_oracle(rt, O):
    """The 32^3 grid, 20,000-line list and 2^15 rays of the full-size
    workload, traced in one call (coherent order, the XCD-major block map over
    two spectral chunks) on the first 3,072 points of its spectral grid, where
    the oracle's kappa of every cell is affordable.  Per cell against the
    oracle."""
    w = I.plain_32cube()
    w = replace(w, lines=replace(w.lines, n_nu=2 * rt.MARCH_CHUNK))
    n = 1 << 15
    t = _tracer(rt, w)
    t.compute_kappa(0)
    _say(f"32^3, {w.lines.n_nu} points: {n} rays in one call")
    t.trace_rays(w.seed, n, 0, n, rt.TALLY_F32)
    got = t.tally()
    assert t.stats()["march_launches"] == 1
    t.close()
    _say(f"  oracle on {oracle_pool.threads()} threads")
    _check_tallies("32^3, 2 chunks, 2^15 rays", got,
                   oracle_pool.run(w.grid, w.lines, n, seed=w.seed))


def test_coherent_order_matches_natural_order(rt):
    """A batch of >= 2^15 rays is marched in the coherent (sorted) order; the
    same rays traced in pieces below that size run in index order.  Only the
    order of the FP64 tally additions may differ."""
    w = I.plain_8cube()
    n = 1 << 16
    t = _tracer(rt, w)
    t.compute_kappa(0)
    _say(f"coherent order: {n} rays in one call")
    t.trace_rays(w.seed, n, 0, n)
    a1, e1, b1 = t.tally()
    t.reset_tally()
    _say("natural order: 4 calls of 2^14 rays")
    for b in range(0, n, 1 << 14):
        t.trace_rays(w.seed, n, b, 1 << 14)
    a2, e2, b2 = t.tally()
    # exact fixed-point sums of the same per-segment values
    assert np.array_equal(a1, a2) and np.array_equal(e1, e2) and np.array_equal(b1, b2)
    t.close()


def test_quadratic_planck_expansion_path(rt, O):
    """With a coarse spectral step the plain march keeps the second-order
    term of its per-lane Planck expansion; tallies still match the oracle."""
    w = I.small_ragged()
    w = I.with_lines(w, dnu=0.05, n_nu=700)
    # relative size of the second-order term over a lane's 15 steps
    c2, span = 1.438776877, 15 * w.lines.dnu
    worst = 0.0
    for T in (w.grid.T.min(), w.grid.T.max()):
        for nu in (w.lines.nu0, w.lines.nu0 + (w.lines.n_nu - 1) * w.lines.dnu):
            th = c2 / T
            r = 1.0 / math.expm1(th * nu)
            g1 = 3.0 / nu - th * (1 + r)
            g2 = -3.0 / nu ** 2 + th * th * r * (1 + r)
            worst = max(worst, 0.5 * abs(g1 * g1 + g2) * span * span)
    assert worst > 2.0 ** -24, "workload must need the quadratic term"
    t = _tracer(rt, w)
    t.compute_kappa(0)
    t.trace_rays(w.seed, w.n_rays)
    ag, eg, _ = t.tally()
    res = O.run(w.grid, w.lines, w.n_rays, seed=w.seed)
    ra = _rel(ag, res["absorbed"])
    re = _rel(eg, res["emitted"])
    _say(f"  quadratic Planck: absorbed max {ra.max():.3e}, emitted {re.max():.3e}")
    assert ra.max() <= REL and re.max() <= REL
    t.close()


def test_coherent_order_across_several_batches(rt):
    """A call larger than one batch of segment scratch (here a 512 x 512 x 1
    grid, ~127k rays per batch) is ordered batch by batch; the tallies equal
    those of the same rays traced in pieces small enough to stay in index
    order."""
    n = 512
    g = I.linear_T_grid(n, 0.01, nz=1, T_lo=400.0, T_hi=1400.0)
    L = I.line_list(40, 1000.0, 1010.0, n_nu=1024)
    w = I.Workload("wide_512x512x1", g, L, 1 << 17, 0)
    t = _tracer(rt, w)
    t.compute_kappa(0)
    _say(f"several batches: {w.n_rays} rays in one call")
    t.trace_rays(w.seed, w.n_rays)
    a1, e1, b1 = t.tally()
    st = t.stats()
    assert st["march_launches"] >= 2, "the call must span several batches"
    t.reset_tally()
    for b in range(0, w.n_rays, 1 << 14):
        t.trace_rays(w.seed, w.n_rays, b, 1 << 14)
    a2, e2, b2 = t.tally()
    assert np.array_equal(a1, a2) and np.array_equal(e1, e2) and np.array_equal(b1, b2)
    t.close()


def test_slab_random_rays_precision_form(rt, O):
    """The 1 m isothermal slab under the precision form with 1,024 random
    boundary rays and hot walls: per-cell tallies and the balance against the
    FP64 oracle."""
    w = I.slab_1cell()
    t = _tracer(rt, w)
    t.compute_kappa(rt.KAPPA_COMPENSATED)
    t.trace_rays(w.seed, w.n_rays, 0, w.n_rays, rt.TALLY_F64)
    ag, eg, bg = t.tally()
    res = O.run(w.grid, w.lines, w.n_rays, seed=w.seed)
    ra = _rel(ag, res["absorbed"])
    re = _rel(eg, res["emitted"])
    rb = _rel(bg, res["balance"])
    _say(f"  slab random rays: absorbed {ra.max():.3e}, emitted {re.max():.3e}, balance {rb.max():.3e}")
    assert ra.max() <= REL and re.max() <= REL and rb.max() <= REL
    t.close()


# ----------------------------------------------------------- degenerate cases
@pytest.mark.parametrize("case", ["no_lines", "no_gas"])
def test_transparent_medium_exact(rt, case):
    """kappa = 0 (an empty line list, or x_H2O = 0 everywhere) with hot walls:
    nothing is absorbed or emitted, and every ray leaves with exactly what it
    brought in."""
    w = I.small_ragged()
    w.grid.T_wall = 1300.0
    if case == "no_lines":
        L = w.lines
        empty = np.zeros(0)
        w = I.with_lines(w, nu=empty, S=empty, gamma=empty, n_T=empty, E_lower=empty)
    else:
        w.grid.x = np.zeros(w.grid.n_cells)
    t = _tracer(rt, w)
    kap, _ = t.compute_kappa(0)
    assert (kap.cpu().numpy() == 0).all()
    t.trace_rays(w.seed, w.n_rays)
    a, e, b = t.tally()
    assert (a == 0).all() and (e == 0).all()
    assert b[0] > 0 and b[1] == 0 and b[2] == 0
    np.testing.assert_allclose(b[3], b[0], rtol=1e-12)
    t.close()


def test_zero_ray_count_is_a_no_op(rt):
    w = I.small_ragged()
    t = _tracer(rt, w)
    t.compute_kappa(0)
    t.trace_rays(w.seed, w.n_rays, 10, 0)
    a, e, b = t.tally()
    assert (a == 0).all() and (e == 0).all() and (b == 0).all()
    t.close()


def test_long_grid_traversal_bit_exact(rt, O):
    """A 1024 x 16 x 16 grid: grazing rays cross hundreds of cells."""
    g = I.linear_T_grid(1024, 0.001, ny=16, nz=16)
    w = I.Workload("long_1024x16x16", g, I.small_ragged().lines, 600, 5)
    t = _tracer(rt, w)
    counts, cells, lens, Og, Dg = t.debug_segments(w.seed, 0, 600)
    Oo, Do, _ = O.rays(w.seed, 0, 600, g.nx, g.ny, g.nz)
    assert (Og == Oo).all() and (Dg == Do).all()
    longest = 0
    for r in range(600):
        c_o, l_o = O.segments(g.nx, g.ny, g.nz, g.cell_m * 100.0, Oo[r], Do[r])
        assert counts[r] == len(c_o)
        assert (cells[r, :counts[r]] == c_o).all()
        np.testing.assert_array_equal(lens[r, :counts[r]], l_o.astype(np.float32))
        longest = max(longest, len(c_o))
    _say(f"  longest traversal {longest} cells")
    assert longest > 100
    t.close()
