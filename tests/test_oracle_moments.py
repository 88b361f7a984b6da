"""Pins of scattered light toward any observer (sect. 4): scattering events
kept as spherical-harmonic moments of their incoming directions, the
Henyey-Greenstein phase function expanded in Legendre terms g^l; and of the
g-factor approximation (isotropic scattering with kappa_sca (1 - g))."""
import math

import numpy as np
import pytest
from scipy.special import eval_legendre

import mcrt_inputs as mi


def unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1)[:, None]


def test_ylm_low_orders_closed_form(orc):
    rng = np.random.default_rng(0)
    for d in unit(rng, 20):
        y = orc.ylm(2, d)
        x, yy, z = d
        c1 = math.sqrt(3 / (4 * math.pi))
        np.testing.assert_allclose(y[0], 0.5 / math.sqrt(math.pi), rtol=1e-15)
        np.testing.assert_allclose(y[1:4], [c1 * yy, c1 * z, c1 * x], rtol=1e-13, atol=1e-15)
        c2 = math.sqrt(15 / (4 * math.pi))
        want = [c2 * x * yy, c2 * yy * z, math.sqrt(5 / (16 * math.pi)) * (3 * z * z - 1),
                c2 * x * z, 0.5 * c2 * (x * x - yy * yy)]
        np.testing.assert_allclose(y[4:9], want, rtol=1e-12, atol=1e-14)


def test_ylm_orthonormal_on_the_sphere(orc):
    """Gauss-Legendre in cos(theta) times the trapezoid rule in phi (exact
    for these degrees)."""
    L = 7
    mu, wmu = np.polynomial.legendre.leggauss(24)
    nphi = 32
    phi = 2 * np.pi * np.arange(nphi) / nphi
    G = np.zeros(((L + 1) ** 2, (L + 1) ** 2))
    for m_, w_ in zip(mu, wmu):
        s = math.sqrt(1 - m_ * m_)
        for p in phi:
            y = orc.ylm(L, [s * math.cos(p), s * math.sin(p), m_])
            G += w_ * (2 * np.pi / nphi) * np.outer(y, y)
    np.testing.assert_allclose(G, np.eye(G.shape[0]), atol=1e-12)


def test_ylm_addition_theorem(orc):
    rng = np.random.default_rng(1)
    a, b = unit(rng, 30), unit(rng, 30)
    L = 10
    for u, v in zip(a, b):
        ya, yb = orc.ylm(L, u), orc.ylm(L, v)
        for l in range(L + 1):
            s = np.dot(ya[l * l:(l + 1) ** 2], yb[l * l:(l + 1) ** 2])
            assert s == pytest.approx((2 * l + 1) / (4 * math.pi) * eval_legendre(l, np.dot(u, v)),
                                      abs=1e-12)


def tail(g, L):
    """Largest phase-function error of the expansion cut after degree L - 1."""
    return sum((2 * l + 1) / (4 * math.pi) * abs(g) ** l for l in range(L, 400))


@pytest.mark.parametrize("g,order", [(0.0, 1), (0.5, 12), (-0.3, 9)])
def test_moments_reproduce_peeloff_sums(orc, g, order):
    """The same run keeps per-view peel-off sums at three views and the
    moments: the moments' sums toward each view match the peel-off sums cell
    by cell within the expansion's cut-off error (exactly for g = 0)."""
    m = mi.cube(n=6, n_packets=6000, tau_v=1.5, nl=8, albedo=0.8, g=g, seed=3)
    views = np.array([[20.0, 10.0], [75.0, 200.0], [140.0, -30.0]])
    idx = np.array([1, 5], np.int32)
    o = orc.Oracle(m, views=views, img_idx=idx, distance=1e20)
    o.run(mode=orc.BW_EPOCH, epoch=10**9, lucy_tau=0.0, sh_order=order)
    assert o.stats["scatters"] > 1000
    sumxi = o.sh[:, 0, :] * 2 * math.sqrt(math.pi)  # sum of xi of a cell's events
    for v, (th, ph) in enumerate(views):
        t, p = math.radians(th), math.radians(ph)
        k = [math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)]
        rec = o.sh_view_sums(k)
        bound = sumxi * tail(g, order) + 1e-12 * np.abs(o.ssca[v]).max()
        assert np.all(np.abs(rec - o.ssca[v]) <= bound)
        assert np.abs(o.ssca[v]).max() > 0


def test_moments_species_asymmetry(orc):
    """Two species with different g at each wavelength: each event carries
    its own species' g^l (the peel-off sums are matched within the cut-off
    error of the larger |g|)."""
    m = mi.torus(n=10, n_clumps=15, n_packets=8000, nl=20, geo_seed=3, pah=False)
    views = np.array([[35.0, 0.0], [80.0, 60.0]])
    idx = np.array([2, 6, 10], np.int32)
    o = orc.Oracle(m, views=views, img_idx=idx, distance=1e20)
    order = 14
    o.run(mode=orc.BW_EPOCH, epoch=10**9, sh_order=order)
    gmax = np.abs(m.g[:, idx]).max()
    sumxi = o.sh[:, 0, :] * 2 * math.sqrt(math.pi)
    for v, (th, ph) in enumerate(views):
        t, p = math.radians(th), math.radians(ph)
        k = [math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)]
        rec = o.sh_view_sums(k)
        assert np.all(np.abs(rec - o.ssca[v]) <= sumxi * tail(gmax, order) +
                      1e-12 * np.abs(o.ssca[v]).max())


def test_gfactor_matches_hg_in_the_diffusion_limit(orc):
    """A thick pure scatterer: in the diffusion limit the packets' path
    lengths depend on kappa_sca only through the transport opacity
    kappa_sca (1 - g), so isotropic scattering at that opacity crosses as many
    cells per packet as Henyey-Greenstein scattering with g (independent
    seeds; within 3 % here, where isotropic scattering at the unreduced
    opacity crosses about 2.4 times as many cells)."""
    g = 0.6
    m = mi.cube(n=10, n_packets=4000, tau_v=60.0, nl=6, albedo=1.0 - 1e-9, g=g, seed=1)
    crossings = {}
    for law, seed in ((orc.SCAT_HG, 21), (orc.SCAT_GFACTOR, 22)):
        o = orc.Oracle(m, scat_law=law)
        o.run(mode=orc.BW_EPOCH, epoch=10**9, lucy_tau=0.0, record=True, seed=seed)
        r = o.records
        assert np.all(r["status"] == orc.ESCAPED)
        crossings[law] = r["n_cross"].astype(float)
        if law == orc.SCAT_GFACTOR:
            # isotropic: about (1 - g) times as many scatterings
            ratio = r["n_scat"].mean() / hg_scat
        else:
            hg_scat = r["n_scat"].mean()
    a, b = crossings[orc.SCAT_HG], crossings[orc.SCAT_GFACTOR]
    assert abs(b.mean() / a.mean() - 1) < 0.03
    assert ratio == pytest.approx(1 - g, rel=0.1)
