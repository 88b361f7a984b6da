"""Pins of oracle parts that the transport tests reach only indirectly.

Each test ties an oracle function to something other than its own formula:
closed-form integrals of the Planck function (Rosseland and Planck means of a
power-law opacity, the grey thin-limit temperature), geometry (which source a
straight escape came from), Philox draws (the emission direction of a packet)
and diffusion theory (mean first-passage time of a sphere).
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy.special import gamma, zeta

import mcrt_inputs as mi

H = 6.62607015e-27
C = 2.99792458e10
K = 1.380649e-16
SIGMA = 2.0 * math.pi ** 5 * K ** 4 / (15.0 * C ** 2 * H ** 3)


def species_model(base, kabs, ksca, g, frac, lam=None):
    """base with per-species opacities constant in wavelength."""
    lam = base.lam_um if lam is None else lam
    nl = lam.size
    return dataclasses.replace(
        base, lam_um=lam, mass_frac=np.asarray(frac, dtype=np.float64),
        kabs=np.array([[k] * nl for k in kabs], dtype=np.float64),
        ksca=np.array([[k] * nl for k in ksca], dtype=np.float64),
        g=np.array([[x] * nl for x in g], dtype=np.float64))


# ------------------------------------------------------------ opacity means

def test_grey_means_equal_the_opacity(orc):
    """Grey opacities: Rosseland mean of the mixture extinction equals the
    mixture extinction and the Planck mean of a species its absorption, at
    any temperature (the weights cancel)."""
    m = species_model(mi.cube(n=4, n_packets=10), [300.0, 50.0], [100.0, 10.0], [0.0, 0.0],
                      [0.4, 0.6])
    o = orc.Oracle(m)
    kext = 0.4 * 400.0 + 0.6 * 60.0
    for T in (15.0, 120.0, 1500.0, 2.0e4):
        assert o.rosseland(T) == pytest.approx(kext, rel=1e-13)
        assert o.planck_mean(0, T) == pytest.approx(300.0, rel=1e-13)
        assert o.planck_mean(1, T) == pytest.approx(50.0, rel=1e-13)


@pytest.mark.parametrize("beta", [1.0, 1.5, 2.0])
def test_power_law_means_closed_form(orc, beta):
    """kappa = k0 (nu/nu0)^beta on a fine grid against the continuous integrals
    int x^(4-b) e^x/(e^x-1)^2 dx = Gamma(5-b) zeta(4-b) (Rosseland, dB/dT
    weights) and int x^(3+b)/(e^x-1) dx = Gamma(4+b) zeta(4+b) (Planck, B
    weights). Using B for dB/dT in the Rosseland weight, or forgetting to
    invert its harmonic sum, changes the result by a factor 1.6-1.8 here."""
    lam = mi.lambda_grid(4000, 1e-3, 1e7)
    nu = C / (lam * 1e-4)
    nu0 = C / 0.55e-4
    k0 = 1.0e3
    kext = k0 * (nu / nu0) ** beta
    base = mi.cube(n=4, n_packets=10)
    m = dataclasses.replace(base, lam_um=lam, mass_frac=np.array([1.0]),
                            kabs=(0.3 * kext)[None, :], ksca=(0.7 * kext)[None, :],
                            g=np.zeros((1, lam.size)))
    o = orc.Oracle(m)
    for T in (30.0, 300.0, 3000.0):
        a = (K * T / (H * nu0)) ** beta
        kr = k0 * a * gamma(5.0) * zeta(4.0) / (gamma(5.0 - beta) * zeta(4.0 - beta))
        kp = 0.3 * k0 * a * gamma(4.0 + beta) * zeta(4.0 + beta) / (gamma(4.0) * zeta(4.0))
        assert o.rosseland(T) == pytest.approx(kr, rel=2e-4)
        assert o.planck_mean(0, T) == pytest.approx(kp, rel=2e-4)


# ------------------------------------------------------------ first guess T

def test_init_T_grey_thin_limit(orc):
    """Grey absorber in the unattenuated field of point sources: the cell
    temperature solves kappa sigma T^4 / pi = kappa sum_s L_s / (16 pi^2 r_s^2),
    i.e. T^4 = sum_s L_s / (16 pi sigma r_s^2). One source, then two."""
    lam = mi.lambda_grid(1500, 1e-2, 1e5)
    base = mi.cube(n=6, n_packets=10)
    m = species_model(base, [200.0], [0.0], [0.0], [1.0], lam=lam)
    half = -base.origin[0]
    for pos, lum in [(np.zeros((1, 3)), np.array([mi.LSUN])),
                     (np.array([[0.1, -0.2, 0.05], [-0.3, 0.25, -0.1]]) * half,
                      np.array([mi.LSUN, 2.5 * mi.LSUN]))]:
        mm = dataclasses.replace(m, src_pos=pos, src_lum=lum,
                                 src_tbb=np.full(lum.size, 5800.0))
        o = orc.Oracle(mm)
        o.init_T()
        n, dc, org = mm.nx, mm.dcell, mm.origin
        idx = np.arange(n)
        # X[c] = (x, y, z) of linear cell c = (iz*n + iy)*n + ix
        zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
        X = np.stack([org[0] + (xx.ravel() + 0.5) * dc, org[1] + (yy.ravel() + 0.5) * dc,
                      org[2] + (zz.ravel() + 0.5) * dc], axis=1)
        t4 = np.zeros(X.shape[0])
        for p, L in zip(pos, lum):
            r2 = np.sum((X - p) ** 2, axis=1)
            t4 += L / (16.0 * math.pi * SIGMA * r2)
        np.testing.assert_allclose(o.T[0], t4 ** 0.25, rtol=2e-5)


# ------------------------------------------------------------ emission draws

def test_source_choice_proportional_to_luminosity(orc):
    """Two sources in an empty grid: every packet leaves in a straight line,
    so its exit point lies on the ray from exactly one source. The share of
    the brighter source (L ratio 1:3) is binomial with p = 3/4."""
    base = mi.cube(n=8, n_packets=20000, seed=11)
    half = -base.origin[0]
    pos = np.array([[-0.3, 0.1, 0.2], [0.25, -0.2, 0.1]]) * half
    m = dataclasses.replace(base, rho=np.zeros_like(base.rho), src_pos=pos,
                            src_lum=np.array([1.0, 3.0]) * mi.LSUN,
                            src_tbb=np.array([5800.0, 3000.0]))
    o = orc.Oracle(m).run(mode=orc.BW_EPOCH, record=True)
    r = o.records
    assert np.all(r["status"] == orc.ESCAPED) and np.all(r["n_cross"] > 0)
    dist = []
    for p in pos:
        v = r["pos"] - p
        along = np.sum(v * r["dir"], axis=1)
        perp = v - along[:, None] * r["dir"]
        dist.append(np.linalg.norm(perp, axis=1) / half + (along < 0) * 1.0)
    dist = np.array(dist)
    on = dist < 1e-9
    assert np.all(on.sum(axis=0) == 1), "each exit lies on exactly one source ray"
    n1 = int(on[1].sum())
    n = r.size
    z = (n1 / n - 0.75) / math.sqrt(0.75 * 0.25 / n)
    assert abs(z) < 4.5, z


def two_species_cube(orc, n_packets, seed=5, tau=0.05):
    base = mi.cube(n=8, n_packets=n_packets, seed=seed, tau_v=tau)
    kv = 1.0e4
    # species 0: kabs 1, ksca 3 (g 0.8); species 1: kabs 3, ksca 1 (g -0.5);
    # equal mass fractions, so the mixture extinction is kv as in the cube
    return species_model(base, [0.25 * kv, 0.75 * kv], [0.75 * kv, 0.25 * kv], [0.8, -0.5],
                         [0.5, 0.5])


def test_absorbing_species_proportional_to_f_kabs(orc):
    """The absorbing species is drawn with probability f_s kabs_s / sum: 1/4
    for species 0 here (its scattering share is 3/4, so swapping the two
    weights would give 3/4)."""
    m = two_species_cube(orc, 100_000, tau=0.5)
    o = orc.Oracle(m).run(mode=orc.BW_EPOCH, lucy_tau=0.0)
    k0, k1 = float(o.k[0].sum()), float(o.k[1].sum())
    n = k0 + k1
    assert n > 20000
    z = (k0 / n - 0.25) / math.sqrt(0.25 * 0.75 / n)
    assert abs(z) < 4.5, z


def test_scattering_species_and_hg_in_transport(orc):
    """Packets with exactly one scattering and nothing else: the incoming
    direction is the emission direction (from the packet's first two Philox
    draws), the outgoing one its escape direction. Their cosine follows the
    mixture sum_s p_s HG(g_s) with p_s = f_s ksca_s / sum = (3/4, 1/4), so
    its mean is 3/4 0.8 + 1/4 (-0.5) = 0.475 (HG mean cosine g; drawing the
    species by kabs instead would give -0.175)."""
    m = two_species_cube(orc, 300_000, seed=7)
    o = orc.Oracle(m).run(mode=orc.BW_EPOCH, record=True)
    r = o.records
    sel = (r["n_scat"] == 1) & (r["n_abs"] == 0) & (r["status"] == orc.ESCAPED)
    assert sel.sum() > 3000
    pid = r["pid"][sel]
    u0 = np.array([orc.draw(m.seed, int(p), 0, 0, 0, 0) for p in pid])
    u1 = np.array([orc.draw(m.seed, int(p), 0, 0, 0, 1) for p in pid])
    phi = 2.0 * math.pi * u0
    mu = 1.0 - 2.0 * u1
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    din = np.stack([s * np.cos(phi), s * np.sin(phi), mu], axis=1)
    cosb = np.sum(din * r["dir"][sel], axis=1)
    mean = cosb.mean()
    e2 = 0.75 * (1 + 2 * 0.64) / 3 + 0.25 * (1 + 2 * 0.25) / 3
    sd = math.sqrt(e2 - 0.475 ** 2) / math.sqrt(cosb.size)
    assert abs(mean - 0.475) < 4.5 * sd, (mean, sd)
    # second moment of the mixture, (1 + 2 g^2)/3 per species
    m2 = np.mean(cosb ** 2)
    assert abs(m2 - e2) < 0.03, (m2, e2)


# ------------------------------------------------------------ MRW deposit

def test_mrw_first_step_deposit(orc):
    """One diffusion step from the centre of a very thick grey cell (the
    packet is stopped after it by an interaction cap of 1). The path length of
    a step has mean rho kappa_R R^2 / 2 (mean exit time R^2/(6D) of a sphere,
    D = c/(3 rho kappa_R)) and relative spread sqrt(1/90)*6; each species
    receives xi rho f_s kappa_P,s l. Grey dust: kappa_R = the mixture
    extinction (not the absorption), kappa_P,s = kabs_s, so the species
    energies stand exactly in the ratio f_0 kabs_0 : f_1 kabs_1."""
    base = mi.cube(n=3, n_packets=20000, seed=3, tau_v=1.0)
    kabs, ksca, frac = [800.0, 200.0], [600.0, 1400.0], [0.3, 0.7]
    m = species_model(base, kabs, ksca, [0.0, 0.0], frac)
    kext = sum(f * (a + s) for f, a, s in zip(frac, kabs, ksca))
    rho = 1000.0 / (kext * m.dcell)  # tau of a cell, face to face = 1000
    m = dataclasses.replace(m, rho=np.full((3, 3, 3), rho))
    o = orc.Oracle(m).run(mode=orc.BW_EPOCH, epoch=10 ** 9, mrw_tau=50.0, mrw_gamma=2.0,
                          max_int=1, lucy_tau=0.0)
    assert o.stats["mrw_steps"] == m.n_packets and o.stats["killed"] == m.n_packets
    xi = o.xi()
    c = 13  # the centre cell holds every deposit
    assert np.count_nonzero(o.epath) == 2 and o.epath[0, c] > 0
    ratio = o.epath[0, c] / o.epath[1, c]
    assert ratio == pytest.approx(frac[0] * kabs[0] / (frac[1] * kabs[1]), rel=1e-12)
    kp = sum(f * a for f, a in zip(frac, kabs))
    ell_mean = o.epath[:, c].sum() / (m.n_packets * xi * rho * kp)
    R = 0.5 * m.dcell
    expect = rho * kext * R * R / 2.0
    sd = expect * 6.0 / math.sqrt(90.0) / math.sqrt(m.n_packets)
    assert abs(ell_mean - expect) < 4.5 * sd, (ell_mean / expect, sd / expect)


# ------------------------------------------------------------ serial B&W

def test_serial_bw_touched_snapshots_equal_full_sweeps(orc):
    """Serial B&W (epoch of one packet) refreshes only the entries touched since
    the last epoch; a run made of one-packet calls (each starts with a sweep
    over every entry) must give the same bits."""
    m = mi.torus(n=10, n_clumps=15, n_packets=400, nl=24)
    a = orc.Oracle(m).run(mode=orc.BW_EPOCH, epoch=1, record=True)
    b = orc.Oracle(m)
    recs = []
    for i in range(m.n_packets):
        b.run(first=i, n=1, mode=orc.BW_EPOCH, epoch=1, record=True, n_total=m.n_packets)
        recs.append(b.records.copy())
    assert np.array_equal(a.k, b.k)
    assert np.array_equal(a.epath, b.epath)
    assert np.array_equal(a.sed, b.sed)
    rb = np.concatenate(recs)
    assert np.array_equal(a.records["dir"], rb["dir"])
    assert np.array_equal(a.records["j"], rb["j"])
