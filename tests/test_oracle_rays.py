"""Pins of the oracle's counter RNG, ray sampling and traversal.

Philox4x64-10 is pinned bit for bit against numpy's independent Philox bit
generator.  The ray law is pinned by its statistics (uniform boundary point,
cosine-weighted direction: E[cos] = 2/3, E[cos^2] = 1/2).  Traversal is
pinned against an independent incremental stepping walk in exact rationals
(a different algorithm from the oracle's sorted plane-crossing list), against
geometric invariants, and against Cauchy's mean-chord formula
E[chord] = 4V/S for uniform, cosine-weighted boundary rays.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O

U = 1 << 21  # fixed-point units per cell edge


# ------------------------------------------------------------------ Philox
@pytest.mark.parametrize("key", [(0, 1), (5, 7), (2**64 - 1, 12345), (0xDEADBEEF, 2**63)])
@pytest.mark.parametrize("ctr", [(0, 0, 0, 0), (17, 3, 0, 0), (2**64 - 1, 0, 0, 0),
                                 (2**64 - 1, 2**64 - 1, 5, 9)])
def test_philox_matches_numpy(key, ctr):
    # numpy's Philox advances its 256-bit counter by one before each block.
    bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(ctr, np.uint64))
    words = bg.random_raw(8)
    c = list(ctr)
    for blk in range(2):
        # increment the 256-bit little-endian counter
        for k in range(4):
            c[k] = (c[k] + 1) % 2**64
            if c[k] != 0:
                break
        got = O.philox(c, key)
        assert [int(x) for x in got] == [int(x) for x in words[4 * blk:4 * blk + 4]]


# ----------------------------------------------------------- ray sampling
def _rays(seed, n, nx, ny, nz):
    return O.rays(seed, 0, n, nx, ny, nz)


def test_ray_origin_on_boundary_odd_in_face():
    nx, ny, nz = 5, 6, 7
    Os, Ds, F = _rays(11, 3000, nx, ny, nz)
    n = np.array([nx, ny, nz])
    for o, d, f in zip(Os, Ds, F):
        a, side = f // 2, f % 2
        assert o[a] == (n[a] * U if side else 0)
        assert (d[a] < 0) if side else (d[a] > 0)
        for t in ((a + 1) % 3, (a + 2) % 3):
            assert o[t] % 2 == 1 and 0 < o[t] < n[t] * U
        r2 = int(d[0]) ** 2 + int(d[1]) ** 2 + int(d[2]) ** 2
        # normal component is floor(sqrt(R^2 - A^2 - B^2)), R = 2^20
        assert (2**20) ** 2 - 2 * abs(int(d[a])) - 1 <= r2 <= (2**20) ** 2


def test_ray_faces_area_weighted():
    nx, ny, nz = 2, 3, 5
    _, _, F = _rays(3, 60000, nx, ny, nz)
    area = np.array([ny * nz, ny * nz, nz * nx, nz * nx, nx * ny, nx * ny], float)
    expect = area / area.sum() * len(F)
    got = np.bincount(F, minlength=6)
    chi2 = ((got - expect) ** 2 / expect).sum()
    assert chi2 < 25.0  # 5 dof, p ~ 1e-4


def test_ray_inface_position_uniform():
    n = 4
    Os, _, F = _rays(21, 40000, n, n, n)
    frac = []
    for o, f in zip(Os, F):
        t1 = (f // 2 + 1) % 3
        frac.append(o[t1] / (n * U))
    frac = np.array(frac)
    hist = np.histogram(frac, bins=16, range=(0, 1))[0]
    expect = len(frac) / 16
    assert ((hist - expect) ** 2 / expect).sum() < 45.0  # 15 dof


def test_ray_direction_cosine_law():
    N = 100000
    Os, Ds, F = _rays(0, N, 8, 8, 8)
    a = F // 2
    Dn = np.abs(Ds[np.arange(N), a]).astype(float)
    norm = np.sqrt((Ds.astype(float) ** 2).sum(1))
    cos = Dn / norm
    # cosine-weighted hemisphere: pdf 2 cos(t) sin(t) dt -> E[cos]=2/3, E[cos^2]=1/2
    for moment, exact, var in ((cos.mean(), 2 / 3, 1 / 2 - 4 / 9), ((cos ** 2).mean(), 1 / 2, 1 / 3 - 1 / 4)):
        assert abs(moment - exact) < 4 * np.sqrt(var / N)
    # azimuth uniform: tangent components have zero mean, equal variance
    t1 = Ds[np.arange(N), (a + 1) % 3].astype(float) / norm
    t2 = Ds[np.arange(N), (a + 2) % 3].astype(float) / norm
    assert abs(t1.mean()) < 4 * np.sqrt(0.25 / N) and abs(t2.mean()) < 4 * np.sqrt(0.25 / N)
    assert abs((t1 ** 2).mean() - 0.25) < 0.01 and abs((t2 ** 2).mean() - 0.25) < 0.01


def test_ray_deterministic_and_seed_dependent():
    o1, d1, f1 = O.ray(0, 77, 8, 8, 8)
    o2, d2, f2 = O.ray(0, 77, 8, 8, 8)
    o3, d3, _ = O.ray(1, 77, 8, 8, 8)
    assert (o1 == o2).all() and (d1 == d2).all() and f1 == f2
    assert not ((o1 == o3).all() and (d1 == d3).all())


# --------------------------------------------------------------- traversal
def _stepping_walk(n, o, d, h_cm):
    """Independent reference: incremental cell-by-cell walk with exact
    rationals.  From the current cell, the next event is the smallest exit
    parameter over the axes; all axes reaching it step together."""
    n = [int(v) for v in n]
    o = [int(v) for v in o]
    d = [int(v) for v in d]
    idx = []
    for k in range(3):
        if o[k] % U == 0:
            idx.append(o[k] // U if d[k] > 0 else o[k] // U - 1)
        else:
            idx.append(o[k] // U)
    t = Fraction(0)
    cells, lens = [], []
    norm = (d[0] ** 2 + d[1] ** 2 + d[2] ** 2) ** 0.5
    while all(0 <= idx[k] < n[k] for k in range(3)):
        tk = []
        for k in range(3):
            if d[k] == 0:
                tk.append(None)
            else:
                bound = (idx[k] + 1) * U if d[k] > 0 else idx[k] * U
                tk.append(Fraction(bound - o[k], d[k]))
        tn = min(v for v in tk if v is not None)
        cells.append(idx[0] + n[0] * (idx[1] + n[1] * idx[2]))
        lens.append((tn - t, norm))
        for k in range(3):
            if tk[k] is not None and tk[k] == tn:
                idx[k] += 1 if d[k] > 0 else -1
        t = tn
    return cells, [float(dt) * nrm * h_cm / U for dt, nrm in lens], t


def _adversarial_rays(n):
    """Rays through edges and corners, axis-parallel rays, shallow grazes."""
    nx, ny, nz = n
    out = []
    # straight through a grid vertex at t = 1: (U, U, U) from (0, 1, 1)
    out.append(((0, 1, 1), (U, U - 1, U - 1)))
    # the main diagonal direction from near a corner: y and z tie all along
    out.append(((0, 3, 3), (1 << 19, 1 << 19, 1 << 19)))
    # edge crossings in x-y only
    out.append(((0, 1, 5 * U // 2 + 1), (U, U - 1, 0)))
    # axis-parallel along each axis
    out.append(((0, U + 1, U + 1), (7, 0, 0)))
    out.append(((U + 1, 0, 2 * U - 1), (0, 1 << 20, 0)))
    out.append(((1, 1, nz * U), (0, 0, -(1 << 20))))
    # from the high faces, through vertices
    out.append(((nx * U, ny * U - 1, ny * U - 1 if nz == ny else nz * U - 1), (-U, -(U - 1), -(U - 1))))
    # grazing: tiny normal component
    out.append(((0, 2 * U + 1, 2 * U + 1), (1, 1 << 20, (1 << 20) - 3)))
    out.append(((0, 2 * U + 1, 2 * U + 1), (1, -(1 << 20), 5)))
    keep = []
    for a, b in out:
        # keep rays whose origin lies on the boundary of this grid
        lim = [nx * U, ny * U, nz * U]
        if all(0 <= a[k] <= lim[k] for k in range(3)) and \
                sum(a[k] in (0, lim[k]) for k in range(3)) >= 1:
            keep.append((np.array(a, np.int64), np.array(b, np.int64)))
    return keep


@pytest.mark.parametrize("n", [(4, 4, 4), (3, 5, 2), (1, 1, 1), (8, 8, 8)])
def test_traversal_matches_stepping_walk(n):
    h_cm = 12.5
    cases = _adversarial_rays(n)
    Os, Ds, _ = O.rays(99, 0, 400, *n)
    cases += list(zip(Os, Ds))
    for o, d in cases:
        cells, lens = O.segments(*n, h_cm, o, d)
        rc, rl, t_exit = _stepping_walk(n, o, d, h_cm)
        assert list(cells) == rc
        np.testing.assert_allclose(lens, rl, rtol=1e-14, atol=0)
        # the cells are distinct and each step moves to a neighbour
        assert len(set(cells.tolist())) == len(cells)
        # total length is the chord |P(t_exit) - O|
        chord = float(t_exit) * np.sqrt((d.astype(float) ** 2).sum()) * h_cm / U
        assert abs(lens.sum() - chord) <= 1e-12 * chord
        assert (lens > 0).all()


def test_traversal_vertex_tie_skips_edge_cells():
    # through the vertex (U, U, U): from cell (0,0,0) straight to (1,1,1)
    cells, lens = O.segments(4, 4, 4, 1.0, np.array([0, 1, 1]), np.array([U, U - 1, U - 1]))
    assert cells[0] == 0 and cells[1] == 1 + 4 * (1 + 4 * 1)


@pytest.mark.parametrize("n", [(4, 4, 4), (2, 3, 6)])
def test_mean_chord_cauchy(n):
    # For uniform, cosine-weighted boundary rays the mean chord is 4V/S.
    N = 40000
    h_cm = 10.0
    Os, Ds, _ = O.rays(5, 0, N, *n)
    tot = np.empty(N)
    for k in range(N):
        _, lens = O.segments(*n, h_cm, Os[k], Ds[k])
        tot[k] = lens.sum()
    nx, ny, nz = n
    V = nx * ny * nz * h_cm ** 3
    S = 2 * h_cm ** 2 * (nx * ny + ny * nz + nz * nx)
    exact = 4 * V / S
    assert abs(tot.mean() - exact) < 4 * tot.std() / np.sqrt(N)
