"""GPU tests of the batched form: many receiver cases in one graph launch,
either per-chunk launches over all cases or one persistent work-queue kernel.

* every case equals its own single-case run bit for bit, in both launch
  shapes (same arithmetic, and the tallies are exact fixed-point sums
  whatever the order of additions);
* every case matches the FP64 oracle: 1e-5 relative per cell, exact zeros;
* graph replays with host work in between reproduce the first launch;
* the autotuner returns a valid tuning, stores it and serves it from the
  cache, and that tuning reproduces the results.
"""
import os

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


def _cases():
    """Uneven cases sharing one line list (ragged spectral length)."""
    base = I.small_ragged()
    L = base.lines
    ws = []
    specs = [((5, 6, 7), 0.1, 700, 0.0, 3), ((4, 4, 4), 0.25, 260, 1400.0, 11),
             ((3, 2, 5), 0.05, 96, 900.0, 5), ((6, 3, 2), 0.15, 1000, 0.0, 8)]
    for (nx, ny, nz), h, nr, Tw, seed in specs:
        g = I.linear_T_grid(nx, h, ny=ny, nz=nz, T_lo=320.0 + seed, T_hi=1650.0, x=0.12, p=1.1,
                            T_wall=Tw)
        g.x = I.rng(seed, I.STREAM_XH2O).uniform(0.03, 0.25, g.n_cells)
        ws.append(I.Workload(f"case_{nx}x{ny}x{nz}", g, L, nr, seed))
    return ws


def _rel(g, o):
    nz = o != 0
    assert (g[~nz] == 0).all()
    return np.abs(g[nz] - o[nz]) / np.abs(o[nz])


def _single(rt, w):
    t = rt.Tracer(0)
    t.setup_grid(w.grid)
    t.setup_lines(w.lines)
    kap, _ = t.alloc_tables()
    t.compute_kappa(rt.KAPPA_PLAIN, kap, None)
    t.trace_rays(w.seed, w.n_rays, 0, w.n_rays, rt.TALLY_F32)
    res = t.tally()
    t.close()
    return res


@pytest.mark.parametrize("mode", ["chunked", "chunked_one_slab", "persistent"])
def test_batch_matches_single_runs_and_oracle(rt, mode):
    from oracle import oracle as O
    cases = _cases()
    t = rt.Tracer(0)
    t.setup_lines(cases[0].lines)
    tun = rt.Tracer.default_tuning()
    tun.mode = rt.BATCH_PERSISTENT if mode == "persistent" else rt.BATCH_CHUNKED
    tun.slots = 1 if mode == "chunked_one_slab" else 2
    tun.chunk_points = rt.MARCH_CHUNK
    tun.kappa_groups = 2
    tun.march_rays = 16
    print("batch prepare", mode, [c.name for c in cases], flush=True)
    ws = t.batch_prepare(cases, rt.KAPPA_PLAIN, tun)
    t.batch_launch()
    out = t.batch_results()
    st = t.stats()
    assert st["batch_updates"] > 0 and st["batch_line_evals"] > 0
    for w, (a, e, b) in zip(cases, out):
        print("  case", w.name, flush=True)
        sa, se, sb = _single(rt, w)
        assert np.array_equal(a, sa) and np.array_equal(e, se) and np.array_equal(b, sb)
        ref = O.run(w.grid, w.lines, w.n_rays, seed=w.seed)
        ra, re_ = _rel(a, ref["absorbed"]), _rel(e, ref["emitted"])
        print(f"    oracle: absorbed max {ra.max():.3e}, emitted max {re_.max():.3e}", flush=True)
        assert ra.max() <= 1e-5 and re_.max() <= 1e-5
        for k in range(4):
            if ref["balance"][k] == 0:
                assert b[k] == 0
            else:
                assert abs(b[k] - ref["balance"][k]) <= 1e-5 * abs(ref["balance"][k])
    t.close()
    del ws


@pytest.mark.parametrize("mode", ["chunked", "persistent"])
def test_batch_compensated_line_sums_match_oracle(rt, mode):
    """The batched launch with compensated line sums (kappa_mode
    RT_KAPPA_COMPENSATED, TwoSum-folded blocks of lines) against the FP64
    oracle per cell and in the balance, and within 1e-5 of the plain
    batched launch (the two differ by the line sums' rounding only)."""
    from oracle import oracle as O
    cases = _cases()
    t = rt.Tracer(0)
    t.setup_lines(cases[0].lines)
    tun = rt.Tracer.default_tuning()
    tun.mode = rt.BATCH_PERSISTENT if mode == "persistent" else rt.BATCH_CHUNKED
    tun.slots = 2
    tun.chunk_points = rt.MARCH_CHUNK
    tun.kappa_groups = 2
    tun.march_rays = 16
    outs, keep = {}, []
    for km in (rt.KAPPA_PLAIN, rt.KAPPA_COMPENSATED):
        print("batch prepare", mode, "kappa mode", km, flush=True)
        keep.append(t.batch_prepare(cases, km, tun))
        t.batch_launch()
        outs[km] = t.batch_results()
    for w, (a, e, b), (ap, ep, bp) in zip(cases, outs[rt.KAPPA_COMPENSATED], outs[rt.KAPPA_PLAIN]):
        ref = O.run(w.grid, w.lines, w.n_rays, seed=w.seed)
        ra, re_ = _rel(a, ref["absorbed"]), _rel(e, ref["emitted"])
        rp = max(_rel(a, ap).max(), _rel(e, ep).max())
        print(f"  {w.name}: oracle absorbed {ra.max():.3e}, emitted {re_.max():.3e}; "
              f"vs plain batched {rp:.3e}", flush=True)
        assert ra.max() <= 1e-5 and re_.max() <= 1e-5 and rp <= 1e-5
        for k in range(4):
            if ref["balance"][k] == 0:
                assert b[k] == 0
            else:
                assert abs(b[k] - ref["balance"][k]) <= 1e-5 * abs(ref["balance"][k])
    t.close()


_SINGLE = {}


@pytest.mark.parametrize("shape", ["committed", "persistent"])
def test_full_64_case_batch_sampled_cases(rt, shape):
    """The 64-case workload (16^3-48^3 cells, 2^14-2^18 rays, 5,000 lines,
    20,000 points) in the launch configuration bench times (the committed
    tuning), and in the persistent launch shape with its own tuning (1,536
    points, 32 groups, 16 rays, 5 blocks per CU, 8 slabs): the smallest, the
    largest and one more case against the single-case path, which is itself
    checked against the oracle."""
    import torch
    cases = I.batched_cases(64)
    t = rt.Tracer(0)
    t.setup_lines(cases[0].lines)
    tun, vals = _committed_tuning(rt)
    if shape == "persistent":
        tun = rt.Tracer.default_tuning()
        (tun.chunk_points, tun.kappa_groups, tun.march_rays, tun.blocks_per_cu, tun.slots) = (
            rt.MARCH_CHUNK, 32, 16, 5, 8)
        tun.mode = rt.BATCH_PERSISTENT
        vals = tun.as_dict()
    print("64-case batch, tuning", vals, flush=True)
    ws = t.batch_prepare(cases, rt.KAPPA_PLAIN, tun)
    t.batch_launch()
    out = t.batch_results()
    t.close()
    del ws
    torch.cuda.empty_cache()
    sizes = [c.grid.n_cells * c.n_rays for c in cases]
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 17})
    for k in pick:
        w = cases[k]
        print(f"  case {k}: {w.grid.nx}^3 cells, {w.n_rays} rays", flush=True)
        if k not in _SINGLE:
            _SINGLE[k] = _single(rt, w)
        sa, se, sb = _SINGLE[k]
        a, e, b = out[k]
        assert np.array_equal(a, sa) and np.array_equal(e, se) and np.array_equal(b, sb)


def _committed_tuning(rt):
    import json
    here = os.path.dirname(os.path.abspath(__file__))
    cache = os.path.join(os.path.dirname(here), "paper_cs_0703028_amd", "tuning", "batch_tune.json")
    vals = list(json.load(open(cache)).values())[0]
    tun = rt.Tracer.default_tuning()
    for (name, _), v in zip(tun._fields_, vals):
        setattr(tun, name, int(v))
    return tun, vals


@pytest.mark.slow
def test_64_case_extremes_match_oracle(rt):
    """The smallest (16^3 cells, 2^14 rays) and the largest (48^3 cells, 2^18
    rays) case of the 64-case workload, with all their rays, its 5,000-line
    list and the committed tuning, batched together on the first 1,000 points
    of the spectral grid (where the oracle's kappa of every cell is
    affordable): per cell and balance against the oracle (rays marched on host
    threads)."""
    from dataclasses import replace
    import oracle_pool
    cases = I.batched_cases(64)
    sizes = [c.grid.n_cells * c.n_rays for c in cases]
    L = replace(cases[0].lines, n_nu=1000)
    pick = [replace(cases[k], lines=L) for k in (int(np.argmin(sizes)), int(np.argmax(sizes)))]
    t = rt.Tracer(0)
    t.setup_lines(L)
    tun, vals = _committed_tuning(rt)
    print("extremes", [c.name for c in pick], "tuning", vals, flush=True)
    ws = t.batch_prepare(pick, rt.KAPPA_PLAIN, tun)
    t.batch_launch()
    out = t.batch_results()
    t.close()
    del ws
    for w, (a, e, b) in zip(pick, out):
        print(f"  {w.name}: oracle on {oracle_pool.threads()} threads", flush=True)
        ref = oracle_pool.run(w.grid, w.lines, w.n_rays, seed=w.seed)
        ra, re_, rb = _rel(a, ref["absorbed"]), _rel(e, ref["emitted"]), _rel(b, ref["balance"])
        print(f"    absorbed max {ra.max():.3e}, emitted max {re_.max():.3e}, balance {rb.max():.3e}",
              flush=True)
        assert ra.max() <= 1e-5 and re_.max() <= 1e-5 and rb.max() <= 1e-5


@pytest.mark.parametrize("mode", ["chunked", "persistent"])
def test_batch_graph_replays(rt, mode):
    cases = _cases()[:3]
    t = rt.Tracer(0)
    t.setup_lines(cases[0].lines)
    tun = rt.Tracer.default_tuning()
    tun.mode = rt.BATCH_CHUNKED if mode == "chunked" else rt.BATCH_PERSISTENT
    tun.slots = 2
    ws = t.batch_prepare(cases, rt.KAPPA_PLAIN, tun)
    t.batch_launch()
    first = t.batch_results()
    for rep in range(3):
        # host work and an unrelated device op between replays
        import torch
        torch.ones(1000, device="cuda").sum().item()
        t.batch_launch()
        again = t.batch_results()
        for (a0, e0, b0), (a1, e1, b1) in zip(first, again):
            assert np.array_equal(a1, a0) and np.array_equal(e1, e0) and np.array_equal(b1, b0)
    t.close()
    del ws


def test_batch_run_one_call(rt):
    # the one-call form (workspace allocated and freed by the library) gives
    # the prepared batch's results, and leaves no batch prepared
    cases = _cases()[:3]
    t = rt.Tracer(0)
    t.setup_lines(cases[0].lines)
    ws = t.batch_prepare(cases)
    t.batch_launch()
    ref = t.batch_results()
    del ws
    got = t.batch_run(cases)
    for (a0, e0, b0), (a1, e1, b1) in zip(ref, got):
        np.testing.assert_allclose(a1, a0, rtol=1e-12, atol=0)
        np.testing.assert_allclose(e1, e0, rtol=1e-12, atol=0)
        np.testing.assert_allclose(b1, b0, rtol=1e-12, atol=0)
    assert t.raw_status("rt_batch_launch") == rt.RT_ESTATE
    t.close()


def test_batch_run_out_of_memory_is_reported(rt):
    # a 2048 x 1 x 1 case with 2^31 rays asks for about 35 TB of segment
    # workspace: the device allocation fails, the call returns RT_ENOMEM,
    # and the handle stays usable
    from dataclasses import replace
    cases = _cases()[:1]
    t = rt.Tracer(0)
    t.setup_lines(cases[0].lines)
    huge = replace(cases[0], grid=I.linear_T_grid(2048, 0.001, ny=1, nz=1), n_rays=1 << 31)
    with pytest.raises(rt.RtError) as e:
        t.batch_run([huge])
    assert e.value.status == rt.RT_ENOMEM
    print("huge batch:", t.last_error(), flush=True)
    assert len(t.batch_run(cases)) == 1
    t.close()


def test_batch_autotune_and_cache(rt, tmp_path):
    import torch
    cases = _cases()
    t = rt.Tracer(0)
    t.setup_lines(cases[0].lines)
    big = rt.Tracer.default_tuning()
    big.chunk_points = 4 * rt.MARCH_CHUNK
    big.blocks_per_cu = 4
    nbytes = t.batch_workspace_size(cases, big)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    path = str(tmp_path / "tune.json")
    print("autotune", flush=True)
    best = t.batch_autotune(cases, rt.KAPPA_PLAIN, ws, path)
    d = best.as_dict()
    assert d["chunk_points"] % rt.MARCH_CHUNK == 0 and d["march_rays"] % 4 == 0
    assert d["mode"] in (rt.BATCH_CHUNKED, rt.BATCH_PERSISTENT)
    assert d["slots"] >= (2 if d["mode"] == rt.BATCH_PERSISTENT else 1)
    assert os.path.exists(path) and '"' in open(path).read()
    best2 = t.batch_autotune(cases, rt.KAPPA_PLAIN, ws, path)
    assert best2.as_dict() == d
    t.batch_prepare(cases, rt.KAPPA_PLAIN, best, ws)
    t.batch_launch()
    out = t.batch_results()
    for w, (a, e, b) in zip(cases[:2], out[:2]):
        sa, se, sb = _single(rt, w)
        assert _rel(a, sa).max() <= 1e-9
    t.close()


def test_batch_errors(rt):
    cases = _cases()[:2]
    t = rt.Tracer(0)
    with pytest.raises(rt.RtError) as e:
        t.batch_prepare(cases)
    assert e.value.status == rt.RT_ESTATE
    t.setup_lines(cases[0].lines)
    bad = rt.Tracer.default_tuning()
    bad.chunk_points = 1000
    with pytest.raises(rt.RtError) as e:
        t.batch_workspace_size(cases, bad)
    assert e.value.status == rt.RT_EINVAL
    bad = rt.Tracer.default_tuning()
    bad.mode = 2
    with pytest.raises(rt.RtError) as e:
        t.batch_workspace_size(cases, bad)
    assert e.value.status == rt.RT_EINVAL
    with pytest.raises(rt.RtError) as e:
        t.batch_launch()
    assert e.value.status == rt.RT_ESTATE
    t.close()
