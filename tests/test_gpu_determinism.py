"""Repeated runs on the GPU are bit-identical: every kappa form, the Planck
table and the traversal (no atomics, fixed summation orders), and the tallies,
which are exact fixed-point integer sums of per-segment values that are
themselves formed in a fixed order, so neither the order in which wavefronts
deliver them nor the way rays are split over calls and launches matters."""
from dataclasses import replace

import numpy as np
import pytest

from paper_cs_0703028_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_cs_0703028_amd import rtlbl
    return rtlbl


def test_kappa_forms_and_traversal_repeat_bit_for_bit(rt):
    w = I.small_ragged()
    t = rt.Tracer(0)
    t.setup_workload(w)
    t.set_line_tolerance(1e-4)
    kap, B = t.alloc_tables()
    for mode in (rt.KAPPA_PLAIN, rt.KAPPA_COMPENSATED, rt.KAPPA_TABLE16, rt.KAPPA_ADAPTIVE):
        t.compute_kappa(mode, kap, B)
        k1, b1 = kap.cpu().numpy().copy(), B.cpu().numpy().copy()
        t.compute_kappa(mode, kap, B)
        assert np.array_equal(k1, kap.cpu().numpy()), mode
        assert np.array_equal(b1, B.cpu().numpy()), mode
    s1 = t.debug_segments(w.seed, 0, 512)
    s2 = t.debug_segments(w.seed, 0, 512)
    for a, b in zip(s1, s2):
        assert np.array_equal(a, b)
    t.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_tallies_repeat_bit_for_bit(rt, prec):
    w = I.plain_8cube()
    t = rt.Tracer(0)
    t.setup_workload(replace(w, grid=replace(w.grid, T_wall=1200.0)))
    t.compute_kappa(rt.KAPPA_PLAIN, *t.alloc_tables())
    runs = []
    for _ in range(3):
        t.reset_tally()
        t.trace_rays(w.seed, w.n_rays, 0, w.n_rays, prec)
        runs.append(t.tally())
    for other in runs[1:]:
        for x, y in zip(runs[0], other):
            assert np.array_equal(x, y)
    assert (runs[0][0] > 0).any()
    t.close()


def test_coherent_order_tallies_repeat_bit_for_bit(rt):
    """2^16 rays in one call run in the coherent order, whose counting-sort
    scatter places rays of one bucket in no fixed order: the tallies are
    still the same bit for bit, and equal those of the same rays traced in
    pieces small enough to run in index order."""
    w = I.plain_8cube()
    n = 1 << 16
    t = rt.Tracer(0)
    t.setup_workload(w)
    t.compute_kappa(rt.KAPPA_PLAIN)
    runs = []
    for _ in range(2):
        t.reset_tally()
        t.trace_rays(w.seed, n, 0, n)
        runs.append(t.tally())
    t.reset_tally()
    for b in range(0, n, 1 << 14):
        t.trace_rays(w.seed, n, b, 1 << 14)
    runs.append(t.tally())
    for other in runs[1:]:
        for x, y in zip(runs[0], other):
            assert np.array_equal(x, y)
    t.close()


@pytest.mark.parametrize("mode", ["chunked", "persistent"])
def test_batched_tallies_repeat_bit_for_bit(rt, mode):
    """Two launches of one prepared batch give the same tallies bit for bit
    (persistent queue: blocks take march items in whatever order they reach
    the queue), and both launch shapes give the same tallies."""
    L = I.small_ragged().lines
    cases = []
    for (nx, ny, nz), h, nr, Tw, seed in (((5, 6, 7), 0.1, 700, 0.0, 3),
                                         ((4, 4, 4), 0.25, 1 << 12, 1400.0, 11),
                                         ((6, 3, 2), 0.15, 1000, 0.0, 8)):
        g = I.linear_T_grid(nx, h, ny=ny, nz=nz, T_lo=320.0 + seed, T_hi=1650.0, x=0.12,
                            p=1.1, T_wall=Tw)
        cases.append(I.Workload(f"case_{nx}x{ny}x{nz}", g, L, nr, seed))
    t = rt.Tracer(0)
    t.setup_lines(cases[0].lines)
    tun = rt.Tracer.default_tuning()
    other = rt.Tracer.default_tuning()
    tun.mode = rt.BATCH_CHUNKED if mode == "chunked" else rt.BATCH_PERSISTENT
    tun.slots = 2
    other.mode = rt.BATCH_PERSISTENT if mode == "chunked" else rt.BATCH_CHUNKED
    other.slots = 2
    ws = t.batch_prepare(cases, rt.KAPPA_PLAIN, tun)
    res = []
    for _ in range(2):
        t.batch_launch()
        res.append(t.batch_results())
    del ws
    ws = t.batch_prepare(cases, rt.KAPPA_PLAIN, other)
    t.batch_launch()
    res.append(t.batch_results())
    for other_res in res[1:]:
        for (a1, e1, b1), (a2, e2, b2) in zip(res[0], other_res):
            assert np.array_equal(a1, a2) and np.array_equal(e1, e2) and np.array_equal(b1, b2)
    del ws
    t.close()
