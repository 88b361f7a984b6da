"""Voxel walk (sect. 2: cell-by-cell flight) against brute-force ray/box
intersection of every cell on tiny grids."""
import numpy as np
import pytest

import mcrt_inputs as mi


def tiny(orc, n=(4, 3, 5), dcell=1.0, origin=(-2.0, -1.5, -2.5)):
    m = mi.cube(n=4, n_packets=10)
    m.nx, m.ny, m.nz = n
    m.origin = np.array(origin, dtype=float)
    m.dcell = dcell
    m.rho = np.ones(n[::-1])
    return orc.Oracle(m)


def brute(o, p0, d):
    """(cell, length) of every cell the ray crosses with positive length."""
    m = o.mi
    segs = []
    for iz in range(m.nz):
        for iy in range(m.ny):
            for ix in range(m.nx):
                lo = m.origin + np.array([ix, iy, iz]) * m.dcell
                hi = lo + m.dcell
                t0, t1 = 0.0, np.inf
                ok = True
                for k in range(3):
                    if d[k] != 0:
                        a, b = (lo[k] - p0[k]) / d[k], (hi[k] - p0[k]) / d[k]
                        t0, t1 = max(t0, min(a, b)), min(t1, max(a, b))
                    elif not (lo[k] <= p0[k] <= hi[k]):
                        ok = False
                if ok and t1 - t0 > 1e-12:
                    segs.append((t0, (iz * m.ny + iy) * m.nx + ix, t1 - t0))
    segs.sort()
    return [s[1] for s in segs], np.array([s[2] for s in segs])


def chord(o, p0, d):
    m = o.mi
    lo, hi = m.origin, m.origin + np.array([m.nx, m.ny, m.nz]) * m.dcell
    t1 = np.inf
    for k in range(3):
        if d[k] > 0:
            t1 = min(t1, (hi[k] - p0[k]) / d[k])
        elif d[k] < 0:
            t1 = min(t1, (lo[k] - p0[k]) / d[k])
    return t1


def check(o, p0, d):
    p0 = np.asarray(p0, float)
    d = np.asarray(d, float)
    d = d / np.linalg.norm(d)
    cells, lens = o.dda(p0, d)
    keep = lens > 1e-12
    bc, bl = brute(o, p0, d)
    assert list(cells[keep]) == bc
    np.testing.assert_allclose(lens[keep], bl, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(lens.sum(), chord(o, p0, d), rtol=1e-12)
    # every step moves one axis by one cell
    m = o.mi
    ijk = np.stack([cells % m.nx, (cells // m.nx) % m.ny, cells // (m.nx * m.ny)], 1)
    assert np.all(np.abs(np.diff(ijk, axis=0)).sum(1) == 1)
    return cells, lens


def test_random_rays(orc):
    o = tiny(orc)
    rng = np.random.default_rng(5)
    for _ in range(200):
        p0 = o.mi.origin + rng.random(3) * np.array([4, 3, 5])
        d = rng.normal(size=3)
        check(o, p0, d)


def test_axis_aligned_and_face_starts(orc):
    o = tiny(orc)
    for d in np.eye(3).tolist() + (-np.eye(3)).tolist():
        check(o, [0.3, 0.2, 0.1], d)
    # start exactly on interior faces / edges / vertex; direction picks the cell
    for p0 in ([0.0, 0.2, 0.1], [0.0, 0.5, 0.1], [0.0, 0.5, 0.5], [1.0, -0.5, 0.5]):
        for d in ([1, 0.3, 0.2], [-1, 0.3, 0.2], [-1, -0.4, -0.7], [0.5, -1, 0.9]):
            check(o, p0, d)


def test_face_rule_start_cell(orc):
    o = tiny(orc)
    cells, _ = o.dda([0.0, 0.5, 0.5], [-1.0, 0.0, 0.0])
    m = o.mi
    # x = 0 is the face between ix = 1 and ix = 2 (origin -2); moving -x starts in ix = 1
    assert cells[0] % m.nx == 1
    cells, _ = o.dda([0.0, 0.5, 0.5], [1.0, 0.0, 0.0])
    assert cells[0] % m.nx == 2


def test_diagonal_through_edges_and_corners(orc):
    o = tiny(orc, n=(4, 4, 4), origin=(-2.0, -2.0, -2.0))
    # exact diagonal from a vertex: ties on all axes at every vertex
    cells, lens = o.dda([-2.0, -2.0, -2.0], np.ones(3) / np.sqrt(3.0))
    assert np.isclose(lens.sum(), 4 * np.sqrt(3.0))
    assert len(cells) == 1 + 3 * 3  # one cell + 3 steps per vertex (two of zero length)
    n = o.mi.nx
    ijk = np.stack([cells % n, (cells // n) % n, cells // (n * n)], 1)
    assert list(ijk[1]) == [1, 0, 0] and list(ijk[2]) == [1, 1, 0]  # x steps first
    check(o, [-2.0, -2.0, -2.0], [1.0, 1.0, 1.0])
    check(o, [-2.0, -1.0, 0.3], [1.0, 1.0, 0.0])
