"""GPU: the path split by wavenumber, as it would shard over several GPUs.

No step of the method couples two spectral points, so G runs over disjoint
spectral ranges (each with only the lines that can reach its range, and the
same Philox rays) must add up to the full run: per-cell absorbed and emitted
power and the four balance terms.  Shards are the 32^3 workload's, with
boundaries on march chunks (so each chunk's points sit in the same lanes as
in the full run), run one after another on this GPU.  The sums are not
bit-identical: a shard's grid starts at its own first point, so each line's
offset from it, and with it kappa and B, round differently in the last
place (measured: 1.4e-10 per cell); the bar is 1e-8.
"""
import numpy as np
import pytest

from paper_cs_0703028_amd import inputs as I

pytestmark = pytest.mark.gpu

N_SHARDS = 8
N_RAYS = 1 << 15   # one trace call of 2^15 rays: the coherent ray order runs


@pytest.fixture(scope="module")
def rt():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_cs_0703028_amd import rtlbl
    return rtlbl


def _run(rt, w):
    t = rt.Tracer(0)
    t.setup_grid(w.grid)
    t.setup_lines(w.lines)
    t.compute_kappa(rt.KAPPA_PLAIN, *t.alloc_tables())
    t.trace_rays(w.seed, N_RAYS)
    a, e, b = t.tally()
    t.close()
    return a, e, b


def test_spectral_shards_add_up_to_the_full_run(rt):
    import torch
    w = I.plain_32cube()
    a0, e0, b0 = _run(rt, w)
    torch.cuda.empty_cache()
    bounds = I.spectral_shard_bounds(w.lines.n_nu, N_SHARDS, rt.lib.rt_march_chunk())
    assert bounds[0][0] == 0 and bounds[-1][1] == w.lines.n_nu
    a1, e1, b1 = np.zeros_like(a0), np.zeros_like(e0), np.zeros_like(b0)
    for lo, hi in bounds:
        s = I.spectral_shard(w, lo, hi)
        print(f"shard [{lo}, {hi}): {len(s.lines.nu)} of {len(w.lines.nu)} lines", flush=True)
        a, e, b = _run(rt, s)
        a1 += a
        e1 += e
        b1 += b
        torch.cuda.empty_cache()
    for name, g, f in (("absorbed", a1, a0), ("emitted", e1, e0)):
        assert np.array_equal(g == 0, f == 0), name
        nz = f > 0
        r = np.abs(g[nz] - f[nz]) / f[nz]
        print(f"{name}: sum of {N_SHARDS} shards vs full run, max rel {r.max():.3e}", flush=True)
        assert r.max() <= 1e-8
    assert np.array_equal(b1 == 0, b0 == 0)   # cold walls: nothing enters
    nz = b0 != 0
    rb = np.abs(b1[nz] - b0[nz]) / np.abs(b0[nz])
    print(f"balance terms: max rel {rb.max():.3e}", flush=True)
    assert rb.max() <= 1e-8
