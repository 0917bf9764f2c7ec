"""rt_trace_rays_noalloc, the trace entry point that allocates nothing,
through the C ABI against rt_trace_rays: the tallies (deterministic fixed-point
sums) must be the same bit for bit.  Two calls in a row share the library's
static device scratch, the second with a smaller input, so stale contents of
the first would show."""
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


def _both(rt, w, n_rays, prec, mode):
    """(rt_trace_rays tallies, rt_trace_rays_noalloc tallies) on one handle."""
    t = rt.Tracer(0)
    t.setup_workload(w)
    t.compute_kappa(mode)
    print(f"{w.name}: {n_rays} rays, prec {prec}: rt_trace_rays", flush=True)
    t.trace_rays(w.seed, n_rays, 0, n_rays, prec)
    ref = t.tally()
    t.reset_tally()
    print(f"{w.name}: {n_rays} rays, prec {prec}: rt_trace_rays_noalloc", flush=True)
    t.trace_rays_noalloc(w.seed, n_rays, 0, n_rays, prec)
    got = t.tally()
    t.close()
    return ref, got


def _same(ref, got):
    for r, g in zip(ref, got):
        assert np.array_equal(r, g)
    assert (ref[0] > 0).any()


def test_noalloc_matches_trace_rays_twice_second_smaller(rt):
    # 2^17 rays on the 32^3 grid fill the 64 MiB scratch about 1.5 times:
    # two batches, each in the coherent ray order
    big = I.plain_32cube()
    _same(*_both(rt, big, 1 << 17, rt.TALLY_F32, rt.KAPPA_PLAIN))
    # then a smaller grid, fewer rays (index order), the precision form
    small = I.small_ragged()
    small.grid.T_wall = 1250.0
    _same(*_both(rt, small, small.n_rays, rt.TALLY_F64, rt.KAPPA_COMPENSATED))


def test_noalloc_ray_subrange_and_errors(rt):
    w = I.plain_8cube()
    t = rt.Tracer(0)
    t.setup_workload(w)
    with pytest.raises(rt.RtError) as e:
        t.trace_rays_noalloc(w.seed, w.n_rays)
    assert e.value.status == rt.RT_ESTATE
    t.compute_kappa(rt.KAPPA_PLAIN)
    t.trace_rays(w.seed, w.n_rays, 100, 300)
    ref = t.tally()
    t.reset_tally()
    t.trace_rays_noalloc(w.seed, w.n_rays, 100, 300)
    _same(ref, t.tally())
    assert t.raw_status("rt_trace_rays_noalloc", 0, 10, 5, 6, 0) == rt.RT_EINVAL
    assert t.raw_status("rt_trace_rays_noalloc", 0, 10, 0, 5, 3) == rt.RT_EINVAL
    t.close()
    # a grid whose traversals do not fit 256 rays in the scratch
    g = I.linear_T_grid(40000, 0.001, ny=1, nz=1)
    L = I.line_list(20, 1000.0, 1004.0, n_nu=400)
    t = rt.Tracer(0)
    t.setup_grid(g)
    t.setup_lines(L)
    kap, _ = t.alloc_tables()
    t.compute_kappa(rt.KAPPA_PLAIN, kap, None)
    with pytest.raises(rt.RtError) as e:
        t.trace_rays_noalloc(0, 100)
    assert e.value.status == rt.RT_EINVAL and "scratch" in t.last_error()
    t.close()
