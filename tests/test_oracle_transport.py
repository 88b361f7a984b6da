"""Pins of the oracle's packet transport (sect. 2, Eqs. 1-5, 10, 15)."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import mcrt_inputs as mi

SIGMA_SB = 5.670374419e-5  # erg/s/cm^2/K^4
H, C, K = 6.62607015e-27, 2.99792458e10, 1.380649e-16


def grey_cube(n=8, tau=1.0, albedo=0.0, g=0.0, nl=12, n_packets=20000):
    m = mi.cube(n=n, n_packets=n_packets, tau_v=tau, nl=nl, albedo=albedo, g=g)
    kabs, ksca, gg = mi.grey_dust(m.lam_um, kext_v=1e4, albedo=albedo, g=g, slope=0.0)
    m.kabs, m.ksca, m.g = kabs, ksca, gg
    return m


# ------------------------------------------------------------ Planck, Eq. 4

def test_planck_stefan_boltzmann(orc):
    lam = np.geomspace(0.01, 1e5, 4000)
    nu, w = orc.freq_grid(lam)
    for T in (30.0, 300.0, 3000.0):
        tot = sum(wj * orc.planck(nj, T) for nj, wj in zip(nu, w))
        assert tot == pytest.approx(SIGMA_SB * T**4 / math.pi, rel=2e-4)


def test_planck_derivative_and_limits(orc):
    for nu in (3e11, 3e13, 3e15):
        for T in (20.0, 500.0, 5000.0):
            h = 1e-5 * T
            fd = (orc.planck(nu, T + h) - orc.planck(nu, T - h)) / (2 * h)
            d = orc.dplanck_dT(nu, T)
            if d > 1e-200:
                assert d == pytest.approx(fd, rel=1e-7)
    assert orc.planck(3e15, 0.0) == 0.0 and orc.planck(3e15, 1.0) == 0.0  # x > 700
    # Rayleigh-Jeans limit 2 nu^2 k T / c^2
    nu, T = 1e8, 1e4
    assert orc.planck(nu, T) == pytest.approx(2 * nu**2 * K * T / C**2, rel=1e-5)


def test_freq_grid_weights_tile_frequency_axis(orc):
    lam = np.geomspace(0.1, 1000.0, 20)
    nu, w = orc.freq_grid(lam)
    r = math.sqrt(lam[1] / lam[0])
    nu_hi, nu_lo = C / (lam[0] / r * 1e-4), C / (lam[-1] * r * 1e-4)
    assert w.sum() == pytest.approx(nu_hi - nu_lo, rel=1e-12)
    assert np.all(w > 0)


def test_temperature_inversion_residual_and_roundtrip(orc):
    m = mi.shell(n=4, n_packets=10)
    m.rho = np.ones((4, 4, 4))
    o = orc.Oracle(m)
    for s in range(2):
        prev = 0.0
        for T in (15.0, 80.0, 400.0, 1500.0, 20000.0):
            phi = o.phi(s, T)
            assert phi > prev
            prev = phi
            Tb = o.invert_T(s, phi)
            assert Tb == pytest.approx(T, rel=1e-11)
            assert abs(o.phi(s, Tb) - phi) <= 1e-10 * phi
    assert o.invert_T(0, 0.0) == 0.0


# ------------------------------------------------------------- emission

def test_emission_isotropic_and_source_spectrum(orc):
    m = grey_cube(n=4, tau=0.0, n_packets=40000)
    m.kabs, m.ksca, m.g = mi.grey_dust(m.lam_um, slope=-1.5)
    m.rho = np.zeros((4, 4, 4))
    o = orc.Oracle(m)
    o.run(record=True)
    r = o.records
    assert np.all(r["status"] == orc.ESCAPED) and np.all(r["n_cross"] > 0)
    d = r["dir"]
    n = len(d)
    assert np.all(np.abs(d.mean(0)) < 5 / np.sqrt(3 * n))
    cov = d.T @ d / n
    assert np.allclose(cov, np.eye(3) / 3, atol=5 * np.sqrt(2 / 15 / n))
    # escape point lies on the box at the straight-line distance from the source
    half = -m.origin[0]
    s = half / np.abs(d).max(1)
    assert np.allclose(r["pos"], s[:, None] * d, rtol=0, atol=1e-9 * half)
    # source wavelength follows w_j L_nu,j of the 5800 K blackbody
    nu, w = orc.freq_grid(m.lam_um)
    p = np.array([wj * orc.planck(nj, 5800.0) for nj, wj in zip(nu, w)])
    p /= p.sum()
    cnt = np.bincount(r["j"], minlength=m.nl)
    ok = p * n > 5
    assert cnt[~ok].sum() <= max(5 * p[~ok].sum() * n, 10)
    chi = stats.chisquare(cnt[ok], p[ok] / p[ok].sum() * cnt[ok].sum())
    assert chi.pvalue > 1e-4


# ---------------------------------------------- tau sampling and Eqs. 2-3

def _tau_path(half, d, rho, kap):
    return rho * kap * half / np.abs(d).max(-1)


def test_first_flight_per_packet(orc):
    """Pure grey absorber, central source: with the interaction cap at one,
    a packet escapes iff tau* > tau to the surface along its direction, and
    otherwise stops at distance tau*/(rho kappa) (Eq. 3)."""
    m = grey_cube(n=8, tau=1.5, albedo=0.0, n_packets=4000)
    o = orc.Oracle(m)
    o.run(record=True, max_int=1, lucy_tau=0.0)
    r = o.records
    rho, kap, half = m.rho.flat[0], m.kabs[0, 0], -m.origin[0]
    tau_star = -np.log([orc.draw(m.seed, int(p), 0, 0, 0, 4) for p in r["pid"]])
    esc = r["status"] == orc.ESCAPED
    kil = r["status"] == orc.KILLED
    assert np.all(esc | kil)
    assert np.all(tau_star[esc] > _tau_path(half, r["dir"][esc], rho, kap))
    pos = r["pos"][kil]
    dist = np.linalg.norm(pos, axis=1)
    np.testing.assert_allclose(dist * rho * kap, tau_star[kil], rtol=1e-10)
    din = pos / dist[:, None]
    assert np.all(tau_star[kil] <= _tau_path(half, din, rho, kap) * (1 + 1e-12))


def test_unscattered_escape_fraction_closed_form(orc):
    """Fraction escaping with no interaction from the centre of a uniform
    cube: (6/4pi) int int exp(-tau_c sqrt(1+u^2+v^2)) (1+u^2+v^2)^-3/2 du dv."""
    tau_c = 1.2
    m = grey_cube(n=8, tau=tau_c, albedo=0.0, n_packets=40000)
    o = orc.Oracle(m)
    o.run(record=True, max_int=1, lucy_tau=0.0)
    frac = np.mean(o.records["status"] == orc.ESCAPED)
    f = lambda v, u: np.exp(-tau_c * np.sqrt(1 + u * u + v * v)) * (1 + u * u + v * v) ** -1.5
    exact = 6 / (4 * np.pi) * integrate.dblquad(f, -1, 1, -1, 1, epsabs=1e-12)[0]
    n = len(o.records)
    assert abs(frac - exact) < 5 * np.sqrt(exact * (1 - exact) / n)


def test_albedo_split(orc):
    A = 0.3
    m = grey_cube(n=8, tau=2.0, albedo=A, n_packets=20000)
    o = orc.Oracle(m)
    o.run(record=True, max_int=1, lucy_tau=0.0)
    r = o.records[o.records["status"] == orc.KILLED]
    k = int(r["n_scat"].sum())
    n = len(r)
    assert r["n_scat"].sum() + r["n_abs"].sum() == n
    assert abs(k / n - A) < 5 * np.sqrt(A * (1 - A) / n)


# ------------------------------------------------------------ HG, Eq. 15

@pytest.mark.parametrize("g", [0.0, 0.3, 0.75, -0.5])
def test_hg_moments_and_normalisation(orc, g):
    u = (np.arange(200000) + 0.5) / 200000
    mu = np.array([orc.hg_mu(g, x) for x in u])
    assert mu.mean() == pytest.approx(g, abs=2e-6)
    assert (mu**2).mean() == pytest.approx((1 + 2 * g * g) / 3, abs=2e-6)
    tot = integrate.quad(lambda x: 2 * np.pi * orc.hg_phase(g, x), -1, 1, epsabs=1e-13)[0]
    mean = integrate.quad(lambda x: 2 * np.pi * x * orc.hg_phase(g, x), -1, 1, epsabs=1e-13)[0]
    assert tot == pytest.approx(1.0, abs=1e-10)
    assert mean == pytest.approx(g, abs=1e-10)
    # the sampled cosines follow the phase function's CDF
    cdf = lambda x: integrate.quad(lambda y: 2 * np.pi * orc.hg_phase(g, y), -1, x)[0]
    samp = mu[:: 997]
    assert stats.kstest(samp, np.vectorize(cdf)).pvalue > 1e-3


def test_scatter_rotation_angle(orc):
    """Pure scatterer, cap at one interaction: the angle between the incoming
    direction (source to scattering point) and the outgoing one is the HG
    cosine of the packet's scattering draw."""
    g = 0.6
    m = grey_cube(n=8, tau=2.0, albedo=1.0, g=g, n_packets=3000)
    o = orc.Oracle(m)
    o.run(record=True, max_int=1, lucy_tau=0.0)
    r = o.records[o.records["status"] == orc.KILLED]
    din = r["pos"] / np.linalg.norm(r["pos"], axis=1)[:, None]
    cosb = np.einsum("ij,ij->i", din, r["dir"])
    # draws: emit 0-3, tau 4, albedo 5, species 6, HG 7, azimuth 8
    mu = np.array([orc.hg_mu(g, orc.draw(m.seed, int(p), 0, 0, 0, 7)) for p in r["pid"]])
    np.testing.assert_allclose(cosb, mu, atol=1e-9)
    np.testing.assert_allclose(np.linalg.norm(r["dir"], axis=1), 1.0, atol=1e-14)


# ------------------------------------------------- re-emission, Eqs. 5, 10

def _chi2_hist(j, p):
    cnt = np.bincount(j, minlength=len(p))
    ok = p * len(j) > 5
    assert cnt[~ok].sum() <= max(5 * p[~ok].sum() * len(j), 10)
    return stats.chisquare(cnt[ok], p[ok] / p[ok].sum() * cnt[ok].sum()).pvalue


def test_reemission_spectrum_frozen(orc):
    m = grey_cube(n=8, tau=3.0, albedo=0.0, nl=30, n_packets=20000)
    m.kabs, m.ksca, m.g = mi.grey_dust(m.lam_um, albedo=0.0, slope=-1.5)
    o = orc.Oracle(m)
    o.T[:] = 600.0
    o.run(record=True, max_int=1, mode=orc.FROZEN, n_iter=1, lucy_tau=0.0)
    # (the run's final Eq. 4 step replaces T; the packets saw 600 K)
    r = o.records[o.records["status"] == orc.KILLED]
    nu, w = orc.freq_grid(m.lam_um)
    p = np.array([w[j] * m.kabs[0, j] * orc.planck(nu[j], 600.0) for j in range(m.nl)])
    assert _chi2_hist(r["j"], p / p.sum()) > 1e-4


def test_reemission_spectrum_bw(orc):
    m = grey_cube(n=8, tau=3.0, albedo=0.0, nl=30, n_packets=20000)
    m.kabs, m.ksca, m.g = mi.grey_dust(m.lam_um, albedo=0.0, slope=-1.5)
    o = orc.Oracle(m)
    o.run(record=True, max_int=1, mode=orc.BW_EPOCH, epoch=10**9, lucy_tau=0.0)
    r = o.records[o.records["status"] == orc.KILLED]
    V = m.dcell**3
    rhs = o.xi() / (4 * np.pi * 1.0 * m.rho.flat[0] * V)
    Tt = o.invert_T(0, rhs)  # one epoch: every cell at E = 0 plus one packet
    nu, w = orc.freq_grid(m.lam_um)
    p = np.array([w[j] * m.kabs[0, j] * orc.dplanck_dT(nu[j], Tt) for j in range(m.nl)])
    assert _chi2_hist(r["j"], p / p.sum()) > 1e-4


# --------------------------------------------- conservation and bookkeeping

def test_energy_conservation_and_counts(orc):
    m = mi.cube(n=16, n_packets=20000, tau_v=3.0)
    o = orc.Oracle(m)
    o.run(mode=orc.BW_EPOCH, epoch=1024)
    st = o.stats
    assert st["escaped"] == m.n_packets and st["killed"] == 0
    assert int(o.sed.sum()) == m.n_packets
    assert int(o.k.sum()) + 0 <= st["absorptions"]
    T = o.finalize()
    E = o.energy()
    V = m.dcell**3
    phi = np.array([o.phi(0, t) if t > 0 else 0.0 for t in T[0]])
    lhs = 4 * np.pi * m.rho.ravel() * V * phi
    assert np.allclose(lhs, E[0], rtol=1e-10, atol=0)


def test_interaction_cap_kills(orc):
    m = mi.cube(n=8, n_packets=2000, tau_v=5.0)
    o = orc.Oracle(m)
    o.run(record=True, max_int=3)
    r = o.records
    kil = r["status"] == orc.KILLED
    assert kil.any()
    assert np.all(r["n_scat"][kil] + r["n_abs"][kil] == 3)
    assert o.stats["killed"] == kil.sum()
    assert int(o.sed.sum()) == (~kil).sum()


def test_resume_is_bitwise(orc):
    m = mi.cube(n=8, n_packets=6000, tau_v=2.0)
    a = orc.Oracle(m).run(mode=orc.BW_EPOCH, epoch=1000)
    b = orc.Oracle(m)
    b.run(first=0, n=3000, mode=orc.BW_EPOCH, epoch=1000, n_total=6000)
    b.run(first=3000, n=3000, mode=orc.BW_EPOCH, epoch=1000, n_total=6000)
    assert np.array_equal(a.k, b.k) and np.array_equal(a.sed, b.sed)
    assert np.array_equal(a.epath, b.epath)


def test_deterministic_repeat(orc):
    m = mi.cube(n=8, n_packets=3000, tau_v=2.0)
    a = orc.Oracle(m).run(record=True)
    b = orc.Oracle(m).run(record=True)
    assert a.records.tobytes() == b.records.tobytes()
