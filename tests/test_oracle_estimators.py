"""Pins of the Lucy estimator (sect. 3.1, Eq. 9), thin equilibrium
temperatures (Eq. 4), the modified random walk (sect. 3.2) and the PAH
two-stage emission (sect. 2.1, Eqs. 6-7)."""
import math

import numpy as np
import pytest
from scipy import stats

import mcrt_inputs as mi


def _gl(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def cell_inv_r2(m, ng=10):
    """(1/V) int_cell dV / (4 pi r^2) for every cell (source at the origin)."""
    x, w = _gl(ng)
    ax = [m.origin[k] + (np.arange(n)[:, None] + 0.5 + 0.5 * x[None, :]) * m.dcell
          for k, n in enumerate((m.nx, m.ny, m.nz))]
    out = np.zeros((m.nz, m.ny, m.nx))
    W = w[:, None, None] * w[None, :, None] * w[None, None, :] / 8.0
    for iz in range(m.nz):
        for iy in range(m.ny):
            for ix in range(m.nx):
                X, Y, Z = np.meshgrid(ax[0][ix], ax[1][iy], ax[2][iz], indexing="ij")
                r2 = X * X + Y * Y + Z * Z
                out[iz, iy, ix] = np.sum(W.transpose(0, 1, 2) * (1 / (4 * np.pi * r2)))
    return out


def test_lucy_dilution_and_thin_temperature(orc):
    """tau_V = 1e-4 cube: every cell is thin, so the absorbed energy is the
    path-length sum: E_i -> xi N rho <kappa_abs> int_cell dV/(4 pi r^2), and
    T_i solves Phi(T) = sum_j w_j kabs_j L_nu,j <1/(4 pi r^2)>_i / (4 pi)."""
    n = 8
    m = mi.cube(n=n, n_packets=200000, tau_v=1e-4)
    o = orc.Oracle(m)
    o.run(mode=orc.BW_EPOCH, epoch=10**9)
    assert o.k.sum() == 0 and o.stats["lucy_deposits"] > 0
    T = o.finalize()[0].reshape(n, n, n)
    g = cell_inv_r2(m)
    nu, w = orc.freq_grid(m.lam_um)
    lnu = np.array([orc.planck(x, 5800.0) for x in nu])
    lnu *= m.src_lum[0] / np.sum(w * lnu)
    E = o.energy()[0].reshape(n, n, n)
    V = m.dcell**3
    expect_E = m.rho * V * np.sum(w * lnu * m.kabs[0]) * g
    # radial shells pool many cells; relative MC error there is well below 1%
    r = np.linalg.norm(np.stack(np.meshgrid(*[np.arange(n) - n / 2 + 0.5] * 3, indexing="ij")), axis=0)
    for lo, hi in ((0, 1.5), (1.5, 2.5), (2.5, 3.5), (3.5, 7)):
        sel = (r >= lo) & (r < hi)
        assert E[sel].sum() / expect_E[sel].sum() == pytest.approx(1.0, rel=0.01)
    # temperatures: one cell per shell; tolerance from the crossing count
    # (about N x solid angle of the cell; T ~ E^(1/5.5) for kappa ~ nu^1.5)
    for idx in [(3, 3, 3), (2, 3, 3), (1, 3, 4), (0, 0, 0)]:
        rhs = np.sum(w * m.kabs[0] * lnu * g[idx]) / (4 * np.pi)
        ncr = m.n_packets * g[idx] * m.dcell**2
        tol = max(4.0 / np.sqrt(ncr) / 5.5, 2e-3)
        assert T[idx] == pytest.approx(o.invert_T(0, rhs), rel=tol)


def test_lucy_off_counts_discrete(orc):
    m = mi.cube(n=8, n_packets=5000, tau_v=1e-4)
    o = orc.Oracle(m).run(lucy_tau=0.0)
    assert o.stats["lucy_deposits"] == 0 and np.all(o.epath == 0)


# ------------------------------------------------------------------ MRW

def theta_form(y):
    """S = 1 - theta_4(y) via the Jacobi imaginary transformation:
    theta_4 = sqrt(pi/a) 2 sum_{n>=0} exp(-pi^2 (n+1/2)^2 / a), y = exp(-a)."""
    a = -math.log(y)
    s = sum(math.exp(-math.pi**2 * (k + 0.5) ** 2 / a) for k in range(200))
    return 1.0 - math.sqrt(math.pi / a) * 2.0 * s


def test_mrw_survival_identity(orc):
    for y in (1e-9, 1e-3, 0.1, 0.5, 0.8, 0.9, 0.95):
        assert orc.mrw_survival(y) == pytest.approx(theta_form(y), rel=1e-12, abs=1e-15)
    assert orc.mrw_survival(1e-12) == pytest.approx(2e-12, rel=1e-9)
    ys = np.linspace(1e-6, 0.97, 400)
    S = np.array([orc.mrw_survival(v) for v in ys])
    # strictly increasing until S rounds to 1 (the alternating sum then
    # carries ~1e-15 absolute rounding; draws never ask beyond 1 - 2^-25)
    core = S < 1 - 1e-9
    assert np.all(np.diff(S[core]) > 0) and np.all(np.diff(S) > -1e-14)


def test_mrw_solve_roundtrip_and_mean_exit(orc):
    for u in (2**-25, 1e-4, 0.3, 0.5, 0.99, 1 - 2**-25):
        y = orc.mrw_solve(u)
        assert orc.mrw_survival(y) == pytest.approx(u, rel=1e-12)
    # <t> = R^2/(6D): with path l = -(3 rho kR R^2 / pi^2) ln y, <l> = rho kR R^2 / 2
    n = 20000
    u = (np.arange(n) + 0.5) / n
    lny = np.log([orc.mrw_solve(x) for x in u])
    mean = np.mean(-3.0 * lny / math.pi**2)
    assert mean == pytest.approx(0.5, rel=2e-4)


def test_mrw_brute_force_walk(orc):
    """Exit path of an isotropic scattering walk (mean free path 1) from the
    centre of a sphere of radius 20: mean and spread follow the diffusion
    law used by the MRW step (R^2/2 in mean free paths, boundary layer
    allowed), and the MRW sampler gives the same distribution shape."""
    rng = np.random.default_rng(1)
    R, n = 20.0, 3000
    paths = np.zeros(n)
    for i in range(n):
        p = np.zeros(3)
        L = 0.0
        while True:
            s = rng.exponential()
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            q = p + s * d
            if q @ q >= R * R:
                b = p @ d
                t = -b + math.sqrt(b * b - (p @ p - R * R))
                L += t
                break
            L += s
            p = q
        paths[i] = L
    # effective radius with the Milne extrapolation length 0.71 mfp
    Re = R + 0.71
    assert paths.mean() == pytest.approx(Re * Re / 2, rel=0.05)
    u = (np.arange(4000) + 0.5) / 4000
    mrw = np.array([-3.0 * math.log(orc.mrw_solve(x)) * Re * Re / math.pi**2 for x in u])
    assert stats.ks_2samp(paths, mrw).pvalue > 1e-3


def test_mrw_in_transport_conserves_packets(orc):
    """Very thick cube (Rosseland optical depth of a cell ~ 10-40): the walk
    fires (cells at 100-200 K have Rosseland depth ~50), every packet still escapes, and it replaces most of the discrete
    interactions of the plain run."""
    m = mi.cube(n=8, n_packets=150, tau_v=1e5, nl=12)
    o = orc.Oracle(m)
    o.run(mode=orc.BW_EPOCH, epoch=100, mrw_tau=8.0, mrw_gamma=2.0, record=True)
    assert o.stats["mrw_steps"] > 0
    assert o.stats["escaped"] == m.n_packets
    off = orc.Oracle(m).run(mode=orc.BW_EPOCH, epoch=100, mrw_tau=0.0)
    assert off.stats["mrw_steps"] == 0 and off.stats["escaped"] == m.n_packets
    n_on = o.stats["absorptions"] + o.stats["scatters"]
    n_off = off.stats["absorptions"] + off.stats["scatters"]
    assert n_on < n_off
    # energy held by the cells stays within a few per cent of the plain run
    T_on, T_off = o.finalize()[0], off.finalize()[0]
    hot = T_off > 0
    assert np.median(T_on[hot] / T_off[hot]) == pytest.approx(1.0, abs=0.15)


# ------------------------------------------------------------------ PAH

def pah_model(n=8, tau=0.02, n_packets=30000):
    m = mi.torus(n=n, n_clumps=20, n_packets=n_packets, nl=40)
    m.rho = np.full((n, n, n), tau / (35000.0 * (-m.origin[0])))
    return m


def test_pah_two_stage_counts(orc):
    m = pah_model()
    o = orc.Oracle(m)
    o.run(mode=orc.BW_EPOCH, epoch=10**9)
    n1 = int(o.kpah.sum())
    assert n1 > 0 and o.stats["pah_stopped"] == n1
    assert o.stats["escaped"] + n1 == m.n_packets
    before = dict(o.stats)
    o.pah_pass(mode=orc.BW_EPOCH, epoch=10**9, record=True)
    assert o.stats["packets"] - before["packets"] == n1
    assert int(o.kpah.sum()) == n1  # pass 2 does not add PAH counts
    assert int(o.sed.sum()) == o.stats["escaped"]


def test_pah_emission_spectrum(orc):
    m = pah_model(tau=1e-3, n_packets=40000)
    o = orc.Oracle(m)
    o.run(mode=orc.BW_EPOCH, epoch=10**9)
    o.pah_pass(mode=orc.BW_EPOCH, epoch=10**9, record=True, max_int=1)
    r = o.records
    esc = r[(r["status"] == orc.ESCAPED) & (r["n_scat"] + r["n_abs"] == 0)]
    nu, w = orc.freq_grid(m.lam_um)
    # rows by absorbed PAH power per unit PAH mass
    V = m.dcell**3
    q = o.kpah * o.xi() / (4 * np.pi * m.mass_frac[2] * m.rho.ravel() * V)
    rows = np.searchsorted(m.pah_edges, q, side="right")
    rows = np.minimum(rows, m.pah_emis.shape[0] - 1)
    cell_rows = np.repeat(rows, o.kpah.astype(np.int64))
    row_of = cell_rows[(esc["pid"] - m.n_packets).astype(np.int64)]
    for rr in np.unique(row_of):
        sel = esc["j"][row_of == rr]
        if len(sel) < 2000:
            continue
        p = w * m.pah_emis[rr]
        p /= p.sum()
        cnt = np.bincount(sel, minlength=m.nl)
        ok = p * len(sel) > 5
        assert stats.chisquare(cnt[ok], p[ok] / p[ok].sum() * cnt[ok].sum()).pvalue > 1e-4
