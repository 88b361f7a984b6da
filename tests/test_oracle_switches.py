"""Pins of the oracle's paper-literal switches: a new optical-depth draw on
entering each cell (the footnote to the sect. 2 interaction test), m
equal-energy source bins emitting n_zyk packets each (Eq. 1), and the
ray-tracer's printed form (Eqs. 13-14: absorption optical depth,
face-to-face cell emission)."""
import numpy as np
import pytest
from scipy import integrate

import mcrt_inputs as mi
from tests.test_oracle_raytrace import D, brute_segments, pixel_rays, small_model
from tests.test_oracle_transport import grey_cube


# ------------------------------------------------- per-cell optical depth

def test_per_cell_draws_brute_force(orc):
    """Pure absorber, interaction cap one. Packet p's flight visits the cells
    of the pinned voxel walk from the source; on entering the k-th one it
    takes draw 4 + k, and it stops in the first cell whose segment depth
    rho kappa l exceeds -ln(draw), at -ln(draw)/(rho kappa) past that
    cell's entry point (Eq. 3 per cell); otherwise it escapes."""
    m = grey_cube(n=6, tau=2.5, albedo=0.0, n_packets=1500)
    rng = np.random.default_rng(5)
    m.rho = m.rho * rng.uniform(0.2, 2.0, m.rho.shape)  # cells of unequal depth
    o = orc.Oracle(m)
    o.run(record=True, max_int=1, lucy_tau=0.0, tau_mode=orc.TAU_PER_CELL)
    r = o.records
    kap = m.kabs[0, 0]
    rhof = m.rho.ravel()
    src = m.src_pos[0]
    n_int = 0
    assert np.all(src == 0.0)
    for rec in r:
        pid = int(rec["pid"])
        # the flight's direction: kept by an escape; for a packet stopped at
        # its first interaction (then re-emitted), the ray to its stop point
        d = rec["dir"] if rec["status"] == orc.ESCAPED else rec["pos"] / np.linalg.norm(rec["pos"])
        cells, lens = o.dda(src, d)
        t, stop = 0.0, None
        for k, (c, ell) in enumerate(zip(cells, lens)):
            ts = -np.log(orc.draw(m.seed, pid, 0, 0, 0, 4 + k))
            if rhof[c] * kap * ell > ts:
                stop = t + ts / (rhof[c] * kap)
                break
            t += ell
        if stop is None:
            assert rec["status"] == orc.ESCAPED
        else:
            n_int += 1
            assert rec["status"] == orc.KILLED
            np.testing.assert_allclose(rec["pos"], src + stop * d, rtol=0,
                                       atol=1e-9 * m.dcell)
    assert 0.2 * len(r) < n_int < 0.98 * len(r)


def test_per_cell_draws_escape_fraction_closed_form(orc):
    """The footnote's claim: a new draw per cell leaves the law of the free
    path unchanged, so the no-interaction escape fraction from the centre of
    a uniform cube is the same double integral as with one draw per flight."""
    tau_c = 1.2
    m = grey_cube(n=8, tau=tau_c, albedo=0.0, n_packets=40000)
    o = orc.Oracle(m)
    o.run(record=True, max_int=1, lucy_tau=0.0, tau_mode=orc.TAU_PER_CELL)
    frac = np.mean(o.records["status"] == orc.ESCAPED)
    f = lambda v, u: np.exp(-tau_c * np.sqrt(1 + u * u + v * v)) * (1 + u * u + v * v) ** -1.5
    exact = 6 / (4 * np.pi) * integrate.dblquad(f, -1, 1, -1, 1, epsabs=1e-12)[0]
    n = len(o.records)
    assert abs(frac - exact) < 5 * np.sqrt(exact * (1 - exact) / n)


def test_per_cell_draws_conserve_and_heat_alike(orc):
    """Whole runs with scattering and re-emission: every packet ends, the
    counts balance, and the per-packet numbers of crossings, scatterings and
    absorptions have the same means as with one draw per flight (same law,
    independent streams: z-tests on the difference of the means)."""
    m = mi.cube(n=8, n_packets=30000, tau_v=3.0, nl=12, seed=2)
    recs = []
    for seed, mode in ((11, orc.TAU_FLIGHT), (12, orc.TAU_PER_CELL)):
        o = orc.Oracle(m)
        o.run(mode=orc.BW_EPOCH, epoch=1 << 40, lucy_tau=0.0, tau_mode=mode, record=True,
              seed=seed)
        st = o.stats
        assert st["escaped"] + st["killed"] == m.n_packets
        assert st["absorptions"] == int(o.k.sum())
        recs.append(o.records)
    for key in ("n_cross", "n_scat", "n_abs"):
        a, b = (r[key].astype(float) for r in recs)
        z = (a.mean() - b.mean()) / np.sqrt(a.var() / a.size + b.var() / b.size)
        assert abs(z) < 4.5, (key, z)


# ------------------------------------------------- stratified source bins

def _cum_source(orc, m):
    """Cumulative source fraction in ascending frequency (descending index):
    c[j] = energy share of bins j..nl-1."""
    nu, w = orc.freq_grid(m.lam_um)
    B = np.array([orc.planck(x, m.src_tbb[0]) for x in nu])
    p = w * B / np.sum(w * B)
    return np.cumsum(p[::-1])[::-1]


def test_stratified_source_bins_fill_equal_energy_strata(orc):
    """N = m n_zyk packets over m strata: the packets whose wavelength lies
    in bins j..nl-1 number N c_j within n_zyk (only the stratum holding the
    boundary is shared), far inside the multinomial spread of plain draws."""
    m_str, nzyk = 2000, 10
    n = m_str * nzyk
    m = grey_cube(n=4, tau=0.0, nl=30, n_packets=n)
    m.rho = np.zeros(m.rho.shape)
    c = _cum_source(orc, m)
    dev = {}
    for strata in (m_str, 0):
        o = orc.Oracle(m)
        o.run(record=True, src_strata=strata)
        j = o.records["j"]
        counts = np.bincount(j, minlength=m.lam_um.size)
        cum = np.cumsum(counts[::-1])[::-1]
        dev[strata] = np.abs(cum - n * c).max()
    assert dev[m_str] <= nzyk
    assert dev[0] > 3 * nzyk


def test_stratified_draw_sits_in_its_stratum(orc):
    """Packet pid's wavelength bin holds the cumulative position
    (pid mod m + u)/m of its own draw u (draw 3 of the emission)."""
    m_str = 37
    m = grey_cube(n=4, tau=0.0, nl=25, n_packets=3000)
    m.rho = np.zeros(m.rho.shape)
    c = _cum_source(orc, m)
    o = orc.Oracle(m)
    o.run(record=True, src_strata=m_str)
    for rec in o.records:
        pid = int(rec["pid"])
        u = (pid % m_str + orc.draw(m.seed, pid, 0, 0, 0, 3)) / m_str
        j = int(rec["j"])
        hi = c[j]
        lo = c[j + 1] if j + 1 < c.size else 0.0
        assert lo - 1e-12 < u <= hi + 1e-12


# ---------------------------------------------- ray-tracer, printed form

def test_literal_slab_along_axis(orc):
    """Viewed along z, each pixel ray crosses nz cells face to face, so the
    printed form of an isothermal absorber sums to the slab solution
    B (1 - exp(-nz tau_cell)), the same as the chord form."""
    m = small_model(n=(4, 4, 5), nl=5, ns=1)
    m.origin = -0.5 * np.array([4, 4, 5], float) * m.dcell
    m.rho = np.full(m.rho.shape, 3e-18)
    m.ksca[:] = 0.0
    idx = np.array([0, 2, 4], np.int32)
    o = orc.Oracle(m, views=np.array([[0.0, 0.0]]), img_idx=idx, distance=D)
    T = np.full((1, 80), 700.0)
    img, _ = o.raytrace(7, 7, T=T, rt_mode=orc.RT_ABS_LITERAL)
    nu, _ = orc.freq_grid(m.lam_um)
    rays, apix = pixel_rays(m, 0.0, 0.0, 7, 7)
    hits = 0
    for ix, iy, r0, d in rays:
        segs = brute_segments(m, r0, d)
        for q, j in enumerate(idx):
            want = 0.0
            if segs:
                want = orc.planck(nu[j], 700.0) * -np.expm1(-5 * 3e-18 * m.kabs[0, j] * m.dcell)
            assert img[0, q, iy, ix] == pytest.approx(apix / D**2 * want, rel=1e-12, abs=1e-300)
        hits += bool(segs)
    assert 0 < hits < 49


def test_literal_brute_force(orc):
    """Oblique views of a two-species model with scattered light: per pixel,
    sum over the cells the ray crosses (brute-force box intersection) of
    [(1 - exp(-rho K dcell)) S_e + Ssca/(dnu dcell^2)] exp(-tau to the
    observer), tau with K = sum_s f_s kabs_s."""
    m = small_model(seed=9)
    nc = m.nx * m.ny * m.nz
    rng = np.random.default_rng(10)
    views = np.array([[33.0, 71.0], [121.0, -40.0]])
    idx = np.array([1, 4], np.int32)
    T = rng.uniform(50, 1500, (2, nc))
    ssca = rng.uniform(0, 1e20, (2, 2, nc))
    rho_rt = m.rho.ravel() * rng.uniform(0.5, 1.5, nc)
    o = orc.Oracle(m, views=views, img_idx=idx, distance=D)
    img, _ = o.raytrace(6, 5, T=T, ssca=ssca, rho_rt=rho_rt, rt_mode=orc.RT_ABS_LITERAL)
    nu, w = orc.freq_grid(m.lam_um)
    K = 0.5 * m.kabs[0] + 0.5 * m.kabs[1]
    rhof = m.rho.ravel()
    for v, (th, ph) in enumerate(views):
        rays, apix = pixel_rays(m, th, ph, 6, 5)
        for ix, iy, r0, d in rays:
            segs = brute_segments(m, r0, d)
            for q, j in enumerate(idx):
                I, tau = 0.0, 0.0
                for _, c, ell in segs:
                    em = sum(0.5 * m.kabs[s, j] * orc.planck(nu[j], T[s, c]) for s in range(2))
                    C = -np.expm1(-rhof[c] * K[j] * m.dcell) * em / K[j]
                    C += ssca[v, q, c] / (w[j] * m.dcell**2)
                    I += C * np.exp(-tau)
                    tau += rho_rt[c] * K[j] * ell
                assert img[v, q, iy, ix] == pytest.approx(apix / D**2 * I, rel=1e-9, abs=1e-300)


def test_literal_thin_cell_luminosity(orc):
    """One thin emitting cell seen face on: the pixels covering its face
    receive (dcell^2 / D^2) rho K dcell B, i.e. its luminosity per steradian
    over D^2 (4 pi rho V K B / (4 pi D^2))."""
    n = 3
    m = small_model(n=(n, n, n), nl=4, ns=1)
    m.origin = -0.5 * n * m.dcell * np.ones(3)
    rho = np.zeros((n, n, n))
    rho[1, 1, 1] = 1e-22
    m.rho = rho
    m.ksca[:] = 0.0
    T = np.full((1, n**3), 900.0)
    npx = 3 * 40
    o = orc.Oracle(m, views=np.array([[0.0, 0.0]]), img_idx=np.array([1, 3], np.int32),
                   distance=D)
    _, sed = o.raytrace(npx, npx, T=T, rt_mode=orc.RT_ABS_LITERAL)
    nu, _ = orc.freq_grid(m.lam_um)
    for q, j in enumerate((1, 3)):
        tau = 1e-22 * m.kabs[0, j] * m.dcell
        want = m.dcell**2 / D**2 * -np.expm1(-tau) * orc.planck(nu[j], 900.0)
        # pixel centres tile the face up to the pixels its edges cut
        assert sed[0, q] == pytest.approx(want, rel=0.06)


def test_literal_adjoint_matches_central_differences(orc):
    m = small_model(n=(4, 4, 4), seed=13, nl=5, lum=3.8e33)
    m.origin = -2.0 * m.dcell * np.ones(3) + np.array([0.3, 0.1, -0.2]) * m.dcell
    nc = 64
    rng = np.random.default_rng(14)
    views = np.array([[25.0, 10.0], [100.0, 200.0]])
    idx = np.array([0, 3], np.int32)
    T = rng.uniform(100, 1200, (2, nc))
    ssca = rng.uniform(0, 1e21, (2, 2, nc))
    npx = npy = 6
    w_img = rng.normal(size=(2, 2, npy, npx))
    w_sed = rng.normal(size=(2, 2))
    rho0 = m.rho.ravel().copy()
    lit = orc.RT_ABS_LITERAL
    o = orc.Oracle(m, views=views, img_idx=idx, distance=D)
    g = o.raytrace_adjoint(npx, npy, w_img=w_img, w_sed=w_sed, T=T, ssca=ssca, rho_rt=rho0,
                           rt_mode=lit)

    def loss(rr):
        img, sed = o.raytrace(npx, npy, T=T, ssca=ssca, rho_rt=rr, rt_mode=lit)
        return np.sum(w_img * img) + np.sum(w_sed * sed)

    fd = np.zeros(nc)
    for c in range(nc):
        h = 1e-4 * rho0[c]
        rp = rho0.copy(); rp[c] += h
        rm = rho0.copy(); rm[c] -= h
        fd[c] = (loss(rp) - loss(rm)) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(fd)
