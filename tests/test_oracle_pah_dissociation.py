"""Pins of PAH photodissociation (sect. 2.1, Eq. 8): the molecules of a cell
dissociate when the energy one of them absorbs within a cooling time reaches
E_crit = N_C/2 eV, and the packets that cell's PAH absorbed in pass 1 then
start from the source as source packets."""
import numpy as np
import pytest
from scipy import stats

from tests.test_oracle_estimators import pah_model

AMU, EV = 1.66053906660e-24, 1.602176634e-12


def pass1(orc, m):
    o = orc.Oracle(m)
    o.run(mode=orc.BW_EPOCH, epoch=10**9)
    assert o.kpah.sum() > 0
    return o


def t_star(o, m, c):
    """Cooling time at which cell c's molecules reach E_crit: N_C/2 eV equals
    the power one molecule absorbs (kpah xi over f rho V / (N_C 12 amu)
    molecules) times t."""
    V = m.dcell**3
    per_gram = o.kpah[c] * o.xi() / (m.mass_frac[m.pah_species] * o.rho.ravel()[c] * V)
    return 0.5 * EV / (12.0 * AMU * per_gram)


def test_threshold_and_independence_of_carbon_number(orc):
    m = pah_model(tau=0.05, n_packets=20000)
    o = pass1(orc, m)
    cells = np.flatnonzero(o.kpah)[:20]
    for c in cells:
        ts = t_star(o, m, c)
        for nc in (20.0, 50.0, 400.0):  # m_PAH and E_crit both scale with N_C
            above = o.pah_dissociates(pah_nc=nc, pah_tcool=ts * (1 + 1e-9))
            below = o.pah_dissociates(pah_nc=nc, pah_tcool=ts * (1 - 1e-9))
            assert above[c] and not below[c]
    none = o.pah_dissociates(pah_nc=50.0, pah_tcool=1e300)
    assert np.array_equal(none, o.kpah > 0)
    assert not o.pah_dissociates(pah_nc=0.0, pah_tcool=1e300).any()


def test_dissociated_cells_emit_from_the_source(orc):
    """Thin model, pass 2 with an interaction cap of one: a packet that leaves
    without interacting flew a straight line from where it was born. Born in
    a dissociating cell, that line passes through the source; otherwise it
    passes through its own cell."""
    m = pah_model(tau=0.2, n_packets=150000)
    o = pass1(orc, m)
    kp = o.kpah.copy()
    busy = np.flatnonzero(kp)
    # a cooling time between two distinct thresholds near the packet-weighted
    # median splits the PAH packets into two sizeable groups
    ts = np.array([t_star(o, m, c) for c in busy])
    order = np.argsort(ts)
    cum = np.cumsum(kp[busy][order]) / kp.sum()
    k = min(np.searchsorted(cum, 0.5), len(order) - 2)
    while ts[order[k + 1]] == ts[order[k]] and k + 2 < len(order):
        k += 1
    tc = np.sqrt(ts[order[k]] * ts[order[k + 1]])
    flag = o.pah_dissociates(pah_nc=50.0, pah_tcool=tc)
    share = kp[flag].sum() / kp.sum()
    assert 0.15 < share < 0.85
    o.pah_pass(mode=orc.BW_EPOCH, epoch=10**9, record=True, max_int=1, pah_nc=50.0,
               pah_tcool=tc)
    r = o.records
    cell_of = np.repeat(np.arange(kp.size), kp.astype(np.int64))[(r["pid"] - m.n_packets).astype(np.int64)]
    direct = (r["status"] == orc.ESCAPED) & (r["n_scat"] + r["n_abs"] == 0)
    src = m.src_pos[0]
    n_src = n_cell = 0
    for rec, c in zip(r[direct], cell_of[direct]):
        p, d = rec["pos"], rec["dir"]
        off = np.linalg.norm(np.cross(p - src, d))
        if flag[c]:
            n_src += 1
            assert off <= 1e-9 * np.linalg.norm(p - src)
            assert np.dot(p - src, d) > 0
        else:
            n_cell += 1
            iz, iy, ix = np.unravel_index(c, (m.nz, m.ny, m.nx))
            lo = m.origin + np.array([ix, iy, iz]) * m.dcell
            hi = lo + m.dcell
            # the line p - t d (t >= 0) meets the cell's box
            t0, t1 = 0.0, np.inf
            for a in range(3):
                if d[a] != 0:
                    u, v = (p[a] - hi[a]) / d[a], (p[a] - lo[a]) / d[a]
                    t0, t1 = max(t0, min(u, v)), min(t1, max(u, v))
            assert t0 <= t1 * (1 + 1e-12)
    assert n_src > 100 and n_cell > 100


def test_all_dissociated_pass_is_a_source_run(orc):
    """With every PAH cell dissociating, pass-2 packets are source packets:
    those that escape without interacting have the same wavelength law as
    the pass-1 source packets that do (two-sample chi^2; the escape
    probability per wavelength is the same for both)."""
    m = pah_model(tau=0.3, n_packets=600000)
    o = orc.Oracle(m)
    o.run(mode=orc.BW_EPOCH, epoch=10**9, record=True, max_int=1)
    r1 = o.records
    j1 = r1["j"][(r1["status"] == orc.ESCAPED) & (r1["n_scat"] + r1["n_abs"] == 0)]
    assert o.kpah.sum() > 0
    o.pah_pass(mode=orc.BW_EPOCH, epoch=10**9, record=True, max_int=1, pah_nc=50.0,
               pah_tcool=1e300)
    r = o.records
    j2 = r["j"][(r["status"] == orc.ESCAPED) & (r["n_scat"] + r["n_abs"] == 0)]
    assert j2.size > 300
    a = np.bincount(j1, minlength=m.nl).astype(float)
    b = np.bincount(j2, minlength=m.nl).astype(float)
    ok = (a + b) > 0
    tab = np.vstack([a[ok], b[ok]])
    keep = tab.sum(axis=0) * b.sum() / (a.sum() + b.sum()) > 5
    assert stats.chi2_contingency(tab[:, keep]).pvalue > 1e-4
