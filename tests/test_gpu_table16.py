"""The paper's 16-point tabulated-profile kappa (RT_KAPPA_TABLE16) through
the C ABI against the FP64 oracle: within 1e-5 relative, exact zeros where
the oracle is zero (the 16-point membership is integer work), every gas."""
from dataclasses import replace

import numpy as np
import pytest

from paper_cs_0703028_amd import inputs as I

pytestmark = pytest.mark.gpu

REL = 1e-5


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


def _rel(g, o):
    nz = o != 0
    assert (g[~nz] == 0).all(), "GPU nonzero where the oracle is exactly zero"
    return np.abs(g[nz] - o[nz]) / np.abs(o[nz])


@pytest.mark.parametrize("wl", ["small_ragged", "plain_8cube", "small_ragged_two_gases"])
def test_table16_kappa_matches_oracle(rt, O, wl):
    w = getattr(I, wl)()
    t = rt.Tracer(0)
    t.setup_workload(w)
    print(f"table16 kappa {wl}", flush=True)
    kap, _ = t.compute_kappa(rt.KAPPA_TABLE16)
    n_nu = w.lines.n_nu
    kg = kap.cpu().numpy().astype(np.float64)
    ko = O.kappa_table16(w.grid, w.lines)
    for g in w.gases:
        ko = ko + O.kappa_table16(replace(w.grid, x=g.x), g.lines)
    assert (kg[:, n_nu:] == 0).all()
    r = _rel(kg[:, :n_nu], ko)
    print(f"  rel err max {r.max():.3e} median {np.median(r):.3e}", flush=True)
    assert r.max() <= REL
    st = t.stats()
    n_lines = len(w.lines.nu) + sum(len(g.lines.nu) for g in w.gases)
    assert st["line_evals"] <= 16 * n_lines * w.grid.n_cells
    t.close()


def test_table16_tallies_match_oracle_march(rt, O):
    w = I.plain_8cube()
    t = rt.Tracer(0)
    t.setup_workload(w)
    t.compute_kappa(rt.KAPPA_TABLE16)
    t.trace_rays(w.seed, w.n_rays, 0, w.n_rays, 0)
    ag, eg, _ = t.tally()
    g = w.grid
    Or, Dr, _ = O.rays(w.seed, 0, w.n_rays, g.nx, g.ny, g.nz)
    kap = O.kappa_table16(g, w.lines)
    a, e, _, _ = O.march(g, w.lines, Or, Dr, O.ray_weight(g, w.lines, w.n_rays), kap,
                         O.planck_rows(g, w.lines))
    ra, re = _rel(ag, a), _rel(eg, e)
    print(f"table16 tallies: absorbed max {ra.max():.3e}, emitted max {re.max():.3e}", flush=True)
    assert ra.max() <= REL and re.max() <= REL
    t.close()


def test_table16_needs_eight_point_cutoff(rt):
    w = I.small_ragged()
    t = rt.Tracer(0)
    t.setup_grid(w.grid)
    t.setup_lines(replace(w.lines, cutoff=5 * w.lines.dnu))
    with pytest.raises(rt.RtError) as e:
        t.compute_kappa(rt.KAPPA_TABLE16)
    assert e.value.status == rt.RT_EUNSUPPORTED
    t.close()


def test_table16_full_size_32cube_sampled_rows(rt, O):
    """The 16-point kappa of the whole 32^3 table (20,000 lines, 50,000
    points), as bench computes it; 64 seeded cells' rows against the oracle."""
    import torch
    w = I.plain_32cube()
    t = rt.Tracer(0)
    t.setup_workload(w)
    kap, _ = t.compute_kappa(rt.KAPPA_TABLE16)
    cells = np.sort(np.random.default_rng(12).choice(w.grid.n_cells, 64, replace=False))
    kg = kap[torch.as_tensor(cells, device=kap.device)].cpu().numpy().astype(np.float64)
    t.close()
    del kap
    torch.cuda.empty_cache()
    n_nu = w.lines.n_nu
    ko = O.kappa_table16(w.grid, w.lines, cells.astype(np.int32))
    assert (kg[:, n_nu:] == 0).all()
    r = _rel(kg[:, :n_nu], ko)
    print(f"table16 32^3 sampled rows: rel err max {r.max():.3e} median {np.median(r):.3e}",
          flush=True)
    assert r.max() <= REL
