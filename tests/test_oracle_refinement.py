"""Pins of one level of refinement (sect. 2: cubes divided into sub-cubes of
their own density): the leaf cells tile the grid, the voxel walk through
them matches brute-force box intersection, and a divided cube whose
sub-cubes keep its density and temperature changes no packet's history,
absorption counts (summed per cube) or image."""
import math

import numpy as np
import pytest

import mcrt_inputs as mi
from tests.test_oracle_raytrace import D, pixel_rays

def refined_cube(n=(4, 3, 5), seed=0, frac=0.45, rmax=3, spread=1.0, tau=1.5):
    m = mi.cube(n=4, n_packets=4000, tau_v=tau, nl=10, seed=seed)
    m.nx, m.ny, m.nz = n
    m.dcell = 1e14
    m.origin = -0.5 * np.array(n, float) * m.dcell + np.array([0.11, -0.07, 0.03]) * m.dcell
    rng = np.random.default_rng(seed)
    m.rho = rng.uniform(0.3, 1.5, n[::-1]) * tau / (1e4 * 2e14)
    return mi.refine_random(m, frac=frac, rmax=rmax, seed=seed, spread=spread)


def leaf_boxes(o):
    out = []
    for leaf in range(o.ncells):
        lo, h, rho = o.leaf_box(leaf)
        if leaf < o.mi.ncells and o.ref[leaf] >= 2:
            continue  # a divided cube is no leaf
        out.append((leaf, lo, h, rho))
    return out


def test_leaves_tile_the_grid(orc):
    m = refined_cube()
    o = orc.Oracle(m)
    boxes = leaf_boxes(o)
    vol = sum(h**3 for _, _, h, _ in boxes)
    assert vol == pytest.approx(m.ncells * m.dcell**3, rel=1e-12)
    assert m.rho_sub.size > 0 and len(boxes) == m.ncells - np.count_nonzero(m.ref) + m.rho_sub.size
    rng = np.random.default_rng(1)
    hi = m.origin + np.array([m.nx, m.ny, m.nz]) * m.dcell
    for x in rng.uniform(m.origin, hi, (300, 3)):
        inside = [l for l, lo, h, _ in boxes if np.all(x >= lo) and np.all(x < lo + h)]
        assert len(inside) == 1
    # sub-cube densities are the ones given, in order
    nc = m.ncells
    assert np.array_equal([o.leaf_box(nc + i)[2] for i in range(m.rho_sub.size)], m.rho_sub)


def brute(o, boxes, p0, d):
    segs = []
    for leaf, lo, h, _ in boxes:
        t0, t1 = 0.0, np.inf
        for a in range(3):
            if d[a] != 0:
                u, v = (lo[a] - p0[a]) / d[a], (lo[a] + h - p0[a]) / d[a]
                t0, t1 = max(t0, min(u, v)), min(t1, max(u, v))
            elif not lo[a] <= p0[a] < lo[a] + h:
                t0, t1 = 1, 0
        if t1 - t0 > 1e-9 * o.mi.dcell:
            segs.append((t0, leaf, t1 - t0))
    segs.sort()
    return segs


def test_walk_through_leaves_brute_force(orc):
    """Rays from random interior points (inside whole and divided cubes),
    and from sub-cube faces, through leaves: the same leaves in order and
    the same lengths as intersecting every leaf box."""
    m = refined_cube(seed=3)
    o = orc.Oracle(m)
    boxes = leaf_boxes(o)
    rng = np.random.default_rng(4)
    hi = m.origin + np.array([m.nx, m.ny, m.nz]) * m.dcell
    starts = list(rng.uniform(m.origin, hi, (60, 3)))
    # points on sub-cube faces of divided cubes
    for leaf in rng.choice(np.arange(m.ncells, o.ncells), 20):
        lo, h, _ = o.leaf_box(leaf)
        p = lo + rng.uniform(0, h, 3)
        p[rng.integers(3)] = lo[rng.integers(3)]
        starts.append(p)
    for p0 in starts:
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        cells, lens = o.dda(p0, d)
        b = [(c, l) for _, c, l in brute(o, boxes, p0, d)]
        got = [(c, l) for c, l in zip(cells, lens) if l > 1e-9 * m.dcell]
        assert [c for c, _ in got] == [c for c, _ in b]
        np.testing.assert_allclose([l for _, l in got], [l for _, l in b], rtol=1e-9,
                                   atol=1e-6 * m.dcell)


def same_density_split(m):
    """Divide cubes but give every sub-cube its cube's density."""
    rho = np.asarray(m.rho).ravel()
    subs = [np.full(int(r) ** 3, rho[c]) for c, r in enumerate(m.ref.ravel()) if r >= 2]
    m2 = mi.ModelInputs(**{**m.__dict__})
    m2.rho_sub = np.concatenate(subs)
    return m2


def cube_totals(o, arr):
    """Per-cube sums of a leaf array (sub-cubes added to their cube)."""
    nc = o.mi.ncells
    out = arr[..., :nc].copy()
    ref = o.ref
    off = 0
    for c in np.flatnonzero(ref >= 2):
        n = int(ref[c]) ** 3
        out[..., c] = arr[..., nc + off: nc + off + n].sum(axis=-1)
        off += n
    return out


def test_split_without_change_keeps_every_history(orc):
    """One draw per flight, temperatures fixed (iterative scheme, one pass):
    dividing cubes into sub-cubes of the same density and temperature leaves
    each packet's events, end point and direction unchanged, and the
    absorption counts of a cube are the sums over its sub-cubes."""
    base = refined_cube(seed=5, frac=0.5, tau=2.0)
    m2 = same_density_split(base)
    plain = mi.ModelInputs(**{**base.__dict__})
    plain.ref = None
    plain.rho_sub = None
    o1 = orc.Oracle(plain)
    o2 = orc.Oracle(m2)
    rng = np.random.default_rng(6)
    T1 = rng.uniform(100, 900, (1, plain.ncells))
    o1.T[:] = T1
    T2 = np.zeros((1, o2.ncells))
    T2[:, :plain.ncells] = T1
    off = 0
    for c in np.flatnonzero(o2.ref >= 2):
        n = int(o2.ref[c]) ** 3
        T2[0, plain.ncells + off: plain.ncells + off + n] = T1[0, c]
        off += n
    o2.T[:] = T2
    kw = dict(mode=orc.FROZEN, n_iter=1, lucy_tau=0.0, record=True)
    o1.run(**kw)
    o2.run(**kw)
    r1, r2 = o1.records, o2.records
    for key in ("status", "j", "n_scat", "n_abs"):
        assert np.array_equal(r1[key], r2[key]), key
    np.testing.assert_allclose(r2["pos"], r1["pos"], rtol=0, atol=1e-6 * base.dcell)
    np.testing.assert_allclose(r2["dir"], r1["dir"], atol=1e-12)
    assert np.all(r2["n_cross"] >= r1["n_cross"]) and r2["n_cross"].sum() > r1["n_cross"].sum()
    assert np.array_equal(cube_totals(o2, o2.k), o1.k)
    assert np.array_equal(o2.sed, o1.sed)


def test_split_without_change_keeps_images(orc):
    base = refined_cube(seed=7, frac=0.5)
    m2 = same_density_split(base)
    plain = mi.ModelInputs(**{**base.__dict__})
    plain.ref = None
    plain.rho_sub = None
    views = np.array([[33.0, 71.0], [121.0, -40.0]])
    idx = np.array([1, 6], np.int32)
    o1 = orc.Oracle(plain, views=views, img_idx=idx, distance=D)
    o2 = orc.Oracle(m2, views=views, img_idx=idx, distance=D)
    rng = np.random.default_rng(8)
    T1 = rng.uniform(100, 900, (1, plain.ncells))
    T2 = np.zeros((1, o2.ncells))
    T2[:, :plain.ncells] = T1
    off = 0
    for c in np.flatnonzero(o2.ref >= 2):
        n = int(o2.ref[c]) ** 3
        T2[0, plain.ncells + off: plain.ncells + off + n] = T1[0, c]
        off += n
    i1, s1 = o1.raytrace(9, 7, T=T1)
    i2, s2 = o2.raytrace(9, 7, T=T2)
    np.testing.assert_allclose(i2, i1, rtol=1e-11, atol=1e-14 * np.abs(i1).max())
    for lit in (orc.RT_ABS_LITERAL,):
        # the printed form counts each cell crossed face to face, so dividing
        # changes it; still finite and positive
        i3, _ = o2.raytrace(9, 7, T=T2, rt_mode=lit)
        assert np.all(np.isfinite(i3)) and i3.max() > 0


def test_refined_brute_force_formal_solution(orc):
    """Images of a refined model with varied sub-cube densities and
    temperatures against the chord-form sum over brute-force leaf segments."""
    m = refined_cube(seed=9, frac=0.5, spread=0.8)
    m.src_lum = np.array([0.0])  # dust emission only
    views = np.array([[40.0, 25.0]])
    idx = np.array([2, 7], np.int32)
    o = orc.Oracle(m, views=views, img_idx=idx, distance=D)
    rng = np.random.default_rng(10)
    T = rng.uniform(50, 1500, (1, o.ncells))
    img, _ = o.raytrace(6, 5, T=T)
    boxes = leaf_boxes(o)
    rho_of = {l: r for l, _, _, r in boxes}
    nu, w = orc.freq_grid(m.lam_um)
    kext = m.kabs[0] + m.ksca[0]
    rays, apix = pixel_rays(m, 40.0, 25.0, 6, 5)
    for ix, iy, r0, d in rays:
        segs = brute(o, boxes, r0, d)
        for q, j in enumerate(idx):
            I, tr = 0.0, 1.0
            for _, c, ell in segs:
                S = m.kabs[0, j] * orc.planck(nu[j], T[0, c]) / kext[j]
                dt = rho_of[c] * kext[j] * ell
                I += tr * S * -np.expm1(-dt)
                tr *= np.exp(-dt)
            assert img[0, q, iy, ix] == pytest.approx(apix / D**2 * I, rel=1e-9, abs=1e-300)


def test_refined_energy_balance_and_mrw(orc):
    """A thick refined cube with B&W, Lucy and diffusion steps: every packet
    ends, the leaf temperatures reproduce the leaf energies (Eq. 4 with each
    leaf's own volume), and diffusion steps happen inside sub-cubes."""
    m = refined_cube(seed=11, frac=0.6, tau=1e5, spread=0.3)
    m.n_packets = 300
    o = orc.Oracle(m)
    o.run(mode=orc.BW_EPOCH, epoch=10**9, mrw_tau=8.0, record=True)
    st = o.stats
    assert st["escaped"] + st["killed"] == m.n_packets and st["killed"] == 0
    assert st["mrw_steps"] > 100
    # some diffusion steps start in sub-cubes
    assert o.epath[0, m.ncells:].max() > 0
    T = o.finalize()
    E = o.energy()
    for leaf in np.flatnonzero(E[0] > 0)[:200]:
        lo, h, rho = o.leaf_box(leaf)
        rhs = E[0, leaf] / (4 * math.pi * m.mass_frac[0] * rho * h**3)
        assert o.phi(0, T[0, leaf]) == pytest.approx(rhs, rel=1e-9)


def refined_pah_model(n=8, seed=12, n_packets=60000, tau=0.3):
    m = mi.torus(n=n, n_clumps=10, n_packets=n_packets, nl=30, geo_seed=seed)
    rng = np.random.default_rng(seed)
    m.rho = rng.lognormal(0.0, 0.7, (n, n, n)) * tau / (35000.0 * (-m.origin[0]))
    return mi.refine_random(m, frac=0.4, rmax=3, seed=seed, spread=0.7)


def test_refined_pah_pass_births_in_leaves(orc):
    """Second PAH stage on a refined grid: a leaf emits its pass-1 count, and
    a pass-2 packet that leaves without interacting flew a straight line
    through the leaf (cube or sub-cube) it was born in."""
    m = refined_pah_model()
    o = orc.Oracle(m)
    o.run(mode=orc.BW_EPOCH, epoch=10**9)
    kp = o.kpah.copy()
    assert kp[m.ncells:].sum() > 50 and kp[:m.ncells].sum() > 50
    o.pah_pass(mode=orc.BW_EPOCH, epoch=10**9, record=True, max_int=1)
    r = o.records
    assert len(r) == kp.sum()
    leaf_of = np.repeat(np.arange(kp.size), kp.astype(np.int64))[(r["pid"] - m.n_packets).astype(np.int64)]
    direct = (r["status"] == orc.ESCAPED) & (r["n_scat"] + r["n_abs"] == 0)
    n_sub = 0
    for rec, leaf in zip(r[direct], leaf_of[direct]):
        lo, h, _ = o.leaf_box(leaf)
        p, d = rec["pos"], rec["dir"]
        t0, t1 = 0.0, np.inf
        for a in range(3):
            if d[a] != 0:
                u, v = (p[a] - lo[a] - h) / d[a], (p[a] - lo[a]) / d[a]
                t0, t1 = max(t0, min(u, v)), min(t1, max(u, v))
        assert t0 <= t1 * (1 + 1e-12)
        n_sub += leaf >= m.ncells
    assert n_sub > 20
