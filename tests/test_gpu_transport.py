"""GPU (HIP, through the C ABI) against the FP64 oracle: packet transport.

FP64 path: per-packet escape point, direction, wavelength and weight within
1e-6 relative and identical event counts; per-cell counts exact; energies and
temperatures within 1e-4 relative (observed ~1e-12)."""
import numpy as np
import pytest

import mcrt_inputs as mi
from tests.pairing import compare_records, gpu_context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    oracle.build(force=False)
    return oracle


def run_pair(orc, m, n=None, first=0, precision="fp64", **kw):
    n = m.n_packets if n is None else n
    o = orc.Oracle(m)
    okw = {k: v for k, v in kw.items() if k in ("mode", "n_iter", "epoch", "lucy_tau", "mrw_tau",
                                                  "mrw_gamma", "max_int", "n_total")}
    o.run(first=first, n=n, record=True, **okw)
    g = gpu_context(m, precision)
    modes = {orc.FROZEN: "frozen", orc.BW_EPOCH: "bw_epoch"}
    gkw = dict(mode=modes[kw.get("mode", orc.BW_EPOCH)], n_iter=kw.get("n_iter", 3),
               epoch_packets=kw.get("epoch", 4096), lucy_tau=kw.get("lucy_tau", 1e-2),
               mrw_tau=kw.get("mrw_tau", 0.0), mrw_gamma=kw.get("mrw_gamma", 2.0),
               max_interactions=kw.get("max_int", 10_000_000), n_total=kw.get("n_total", m.n_packets),
               record=True)
    st = g.run_packets(first=first, n=n, seed=m.seed, **gkw)
    return o, g, st


def check_cells(o, g, rtol=1e-4):
    k, ep, kp = g.tallies()
    assert np.array_equal(k, o.k), "absorption counts differ"
    assert np.array_equal(kp, o.kpah), "PAH counts differ"
    scale = max(np.abs(o.epath).max(), 1e-300)
    np.testing.assert_allclose(ep, o.epath, rtol=rtol, atol=1e-12 * scale)
    fl, cnt = g.sed()
    assert np.array_equal(cnt, o.sed), "SED counts differ"


@pytest.mark.parametrize("mode", ["bw_epoch", "frozen"])
def test_cube_fp64_per_packet(orc, mode):
    """32^3 cube, 5800 K star, tau_V = 1, albedo 0.5, g = 0.5, 1e5 packets."""
    m = mi.cube(n=32, n_packets=100_000)
    o = orc.Oracle(m)
    g = gpu_context(m)
    if mode == "frozen":
        o.init_T()
        g.init_temperatures()
        o.run(record=True, mode=orc.FROZEN, n_iter=2)
        st = g.run_packets(0, m.n_packets, m.seed, mode="frozen", n_iter=2, record=True,
                           n_total=m.n_packets)
    else:
        o.run(record=True, mode=orc.BW_EPOCH, epoch=4096)
        st = g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=4096,
                           record=True, n_total=m.n_packets)
    info = compare_records(g.records(m.n_packets), o.records, tol=1e-6, scale=-m.origin[0])
    print(mode, info, flush=True)
    check_cells(o, g)
    To = o.finalize() if mode == "bw_epoch" else o.T
    np.testing.assert_allclose(g.temperatures(), To, rtol=1e-4, atol=0)
    for key in ("escaped", "killed", "scatters", "absorptions", "crossings"):
        assert st[key] == o.stats[key], key


def test_init_temperatures(orc):
    """Thin-limit first guess of the iterative scheme, cell by cell."""
    m = mi.shell(n=24, n_packets=10)
    o = orc.Oracle(m)
    o.init_T()
    g = gpu_context(m)
    g.init_temperatures()
    np.testing.assert_allclose(g.current_temperatures(), o.T, rtol=1e-11, atol=0)


@pytest.mark.parametrize("method,tol", [(0, 1e-12), (1, 1e-9)])
def test_eq4_inversion_matches_oracle(orc, method, tol):
    """Device Eq. 4 (Newton, and the Hermite table used at every immediate
    B&W absorption) against the oracle's bisection, 3 K .. 3e4 K."""
    m = mi.torus(n=8, n_clumps=5, n_packets=10)
    o = orc.Oracle(m)
    g = gpu_context(m)
    for s in (0, 1):
        Ts = np.geomspace(3.5, 3e4, 400)
        rhs = np.array([o.phi(s, t) for t in Ts])
        got = g.invert_temperature(s, rhs, method)
        ref = np.array([o.invert_T(s, r) for r in rhs])
        np.testing.assert_allclose(got, ref, rtol=tol)
        np.testing.assert_allclose(got, Ts, rtol=max(tol, 1e-11))
    # outside the table both fall back or clamp like the oracle
    lo = g.invert_temperature(0, np.array([o.phi(0, 1.5), 0.0, o.phi(0, 2e5)]), method)
    assert lo[0] == pytest.approx(1.5, rel=1e-9) and lo[1] == 0.0 and lo[2] == 1e5


def test_resume_and_determinism(orc):
    m = mi.cube(n=16, n_packets=20000, tau_v=2.0)
    a = gpu_context(m)
    a.run_packets(0, 20000, 0, mode="bw_epoch", epoch_packets=1000, n_total=20000)
    b = gpu_context(m)
    b.run_packets(0, 12000, 0, mode="bw_epoch", epoch_packets=1000, n_total=20000)
    b.run_packets(12000, 8000, 0, mode="bw_epoch", epoch_packets=1000, n_total=20000)
    ka, ea, _ = a.tallies()
    kb, eb, _ = b.tallies()
    assert np.array_equal(ka, kb)
    np.testing.assert_allclose(ea, eb, rtol=1e-12)
    assert np.array_equal(a.sed()[1], b.sed()[1])
    # queue depth and launch shape do not change the result
    c = gpu_context(m)
    c.run_packets(0, 20000, 0, mode="bw_epoch", epoch_packets=1000, n_total=20000,
                  queue_depth=64, walk_blocks_per_cu=1, blocks_per_cu=1)
    assert np.array_equal(ka, c.tallies()[0])


def test_lucy_thin_cube(orc):
    m = mi.cube(n=16, n_packets=30000, tau_v=1e-3)
    o, g, st = run_pair(orc, m, mode=orc.BW_EPOCH, epoch=8192)
    assert o.stats["lucy_deposits"] > 0
    compare_records(g.records(m.n_packets), o.records, scale=-m.origin[0])
    check_cells(o, g)


def test_mrw_thick_cube(orc):
    """Modified random walk in a very thick cube. A walk step moves the
    packet by the distance to the nearest face, p -> p + R(p) d_s, whose
    Jacobian I + d_s n^T makes long chains amplify last-bit differences of
    exp/log between the two codes (measured: identical to 1e-9 relative up
    to ~2000 events, then ~20x per 1000 events). Per-packet parity is
    therefore checked on chains cut at 1500 interactions, with one epoch so
    packets do not couple through energy snapshots; the full run is
    compared statistically."""
    m = mi.cube(n=8, n_packets=150, tau_v=1e5, nl=12)
    o, g, st = run_pair(orc, m, mode=orc.BW_EPOCH, epoch=10**9, mrw_tau=8.0, mrw_gamma=2.0,
                        max_int=1500)
    assert o.stats["mrw_steps"] > 1000 and st["mrw_steps"] == o.stats["mrw_steps"]
    compare_records(g.records(m.n_packets), o.records, scale=-m.origin[0])
    check_cells(o, g, rtol=1e-9)
    # full chains: same physics within Monte Carlo noise
    o2 = orc.Oracle(m).run(mode=orc.BW_EPOCH, epoch=100, mrw_tau=8.0, mrw_gamma=2.0)
    g2 = gpu_context(m)
    s2 = g2.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=100, mrw_tau=8.0,
                        mrw_gamma=2.0, n_total=m.n_packets)
    assert s2["escaped"] == m.n_packets
    assert s2["mrw_steps"] == pytest.approx(o2.stats["mrw_steps"], rel=0.15)
    k2, ep2, _ = g2.tallies()
    assert ep2.sum() == pytest.approx(o2.epath.sum(), rel=0.15)


def test_interaction_cap(orc):
    m = mi.cube(n=8, n_packets=3000, tau_v=5.0)
    o, g, st = run_pair(orc, m, mode=orc.BW_EPOCH, max_int=3)
    assert st["killed"] == o.stats["killed"] > 0
    compare_records(g.records(m.n_packets), o.records, scale=-m.origin[0])


def test_pah_two_stage(orc):
    n = 16
    m = mi.torus(n=n, n_clumps=30, n_packets=20000, nl=40)
    o = orc.Oracle(m)
    o.run(mode=orc.BW_EPOCH, epoch=5000, record=True)
    g = gpu_context(m)
    g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=5000, record=True,
                  n_total=m.n_packets)
    compare_records(g.records(m.n_packets), o.records, scale=-m.origin[0])
    npah = int(o.kpah.sum())
    assert npah > 0
    o.pah_pass(mode=orc.BW_EPOCH, epoch=5000, record=True)
    st = g.run_pah(m.seed, mode="bw_epoch", epoch_packets=5000, record=True)
    assert st["packets"] == npah
    compare_records(g.records(npah), o.records, scale=-m.origin[0])
    check_cells(o, g)


def test_voxelize_torus_and_shell_match(orc):
    """Torus cells are decided by exact FP64 comparisons: bit-identical.
    Shell cell averages agree to rounding."""
    m = mi.torus(n=48, n_clumps=300, n_packets=10)
    g = gpu_context(m)
    ref = orc.voxelize_torus(m.nx, m.ny, m.nz, m.origin, m.dcell, m.geometry)
    assert np.array_equal(g.density(), ref.ravel())
    g32 = gpu_context(m, "fp32")
    assert np.array_equal(g32.density(), ref.ravel().astype(np.float32))
    s = mi.shell(n=24, n_packets=10)
    gs = gpu_context(s)
    refs = orc.voxelize_shell(s.nx, s.ny, s.nz, s.origin, s.dcell, s.geometry)
    np.testing.assert_allclose(gs.density(), refs.ravel(), rtol=1e-12, atol=0)


def test_fp32_first_flight_and_aggregates(orc):
    """FP32 walk: the first emission draws give the same direction and
    wavelength as the FP64 oracle at the same seed. Aggregates are compared
    with an oracle run at an independent seed, so the two noises are
    independent and the chi^2 / z normalisations hold."""
    m = mi.cube(n=32, n_packets=200_000, tau_v=1.0)
    o = orc.Oracle(m)
    o.run(mode=orc.BW_EPOCH, epoch=4096, record=True)
    g = gpu_context(m, "fp32")
    g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=4096, record=True,
                  n_total=m.n_packets)
    rg = g.records(m.n_packets)
    # packets with no interaction keep their emission direction
    free = (o.records["n_scat"] + o.records["n_abs"] == 0) & (rg["n_scat"] + rg["n_abs"] == 0)
    assert free.mean() > 0.2
    np.testing.assert_allclose(rg["dir"][free], o.records["dir"][free], atol=2e-6)
    assert np.mean(rg["j"][free] == o.records["j"][free]) > 0.9999
    # aggregates against an independent oracle sample
    oi = orc.Oracle(m)
    oi.run(mode=orc.BW_EPOCH, epoch=4096, seed=m.seed + 1000)
    so, sg = oi.sed.astype(float), g.sed()[1].astype(float)
    ok = (so + sg) > 50
    chi = np.sum((so[ok] - sg[ok]) ** 2 / (so[ok] + sg[ok])) / ok.sum()
    assert chi < 1.4, chi
    T = g.temperatures()[0]
    To = oi.finalize()[0]
    k, kg = oi.k[0].astype(float), g.tallies()[0][0].astype(float)
    sel = (k > 30) & (kg > 30)
    assert sel.sum() > 150
    z = (T[sel] / To[sel] - 1) / (np.sqrt(1 / k[sel] + 1 / kg[sel]) / 5.5)
    assert np.mean(np.abs(z) < 4) > 0.97
    assert abs(np.median(z)) < 0.5


def test_ticket_mode_statistics(orc):
    """Immediate B&W (GPU order) against the oracle's serial B&W at an
    independent seed."""
    m = mi.cube(n=8, n_packets=100_000, tau_v=3.0)
    o = orc.Oracle(m).run(mode=orc.BW_EPOCH, epoch=1, seed=m.seed + 777)
    g = gpu_context(m)
    g.run_packets(0, m.n_packets, m.seed, mode="bw_ticket", n_total=m.n_packets)
    To = o.finalize()[0]
    T = g.temperatures()[0]
    k, kg = o.k[0].astype(float), g.tallies()[0][0].astype(float)
    sel = (k > 100) & (kg > 100)
    assert sel.sum() > 50
    z = (T[sel] / To[sel] - 1) / (np.sqrt(1 / k[sel] + 1 / kg[sel]) / 5.5)
    assert np.mean(np.abs(z) < 4) > 0.97
    assert abs(np.median(z)) < 0.5
    so, sg = o.sed.astype(float), g.sed()[1].astype(float)
    ok = (so + sg) > 50
    assert np.sum((so[ok] - sg[ok]) ** 2 / (so[ok] + sg[ok])) / ok.sum() < 1.4


def test_fp32_walk_through_empty_bricks():
    """FP32 walk across bricks with no dust: the walk skips their density
    loads (occupancy bits) but must step through them exactly as through
    dust-filled ones. Two grids differ only in 4^3 blocks that are empty in
    one and hold a negligible density (tau ~ 1e-18 per cell) in the other; no
    packet interacts, so the crossing totals and the escape SED must be
    identical. The grid is not cubic and its sizes are not multiples of the
    brick side."""
    import dataclasses
    m = mi.cube(n=8, n_packets=20_000)
    nx, ny, nz = 37, 29, 45
    dc = m.dcell
    origin = -0.5 * dc * np.array([nx, ny, nz], dtype=np.float64) + 0.37 * dc
    rng = np.random.default_rng(12)
    box = rng.random(((nz + 3) // 4, (ny + 3) // 4, (nx + 3) // 4)) < 0.5
    occ = np.repeat(np.repeat(np.repeat(box, 4, 0), 4, 1), 4, 2)[:nz, :ny, :nx]
    tiny = 1e-35
    rho_gaps = np.where(occ, tiny, 0.0)
    rho_full = np.full((nz, ny, nx), tiny)
    out = []
    for rho in (rho_gaps, rho_full):
        mm = dataclasses.replace(m, name="gaps", nx=nx, ny=ny, nz=nz, origin=origin, rho=rho)
        g = gpu_context(mm, "fp32")
        st = g.run_packets(0, mm.n_packets, mm.seed, mode="bw_ticket", n_total=mm.n_packets)
        out.append((st, g.sed()[1].copy()))
    (sa, ea), (sb, eb) = out
    assert sa["escaped"] == sb["escaped"] == m.n_packets
    assert sa["crossings"] == sb["crossings"]
    assert sa["crossings"] > 15 * m.n_packets
    np.testing.assert_array_equal(ea, eb)


def test_sed_flux_of_a_bare_source(orc):
    """Photon-counting SED (sect. 4) of a blackbody source in an empty grid:
    every packet escapes unscattered, so in each polar bin and wavelength the
    flux count xi / (dOmega D^2 w_j) is L_nu,j / (4 pi D^2) within the
    bin's Poisson error (the source spectrum normalised to the luminosity on
    the frequency quadrature)."""
    m = mi.cube(n=8, n_packets=400_000, tau_v=1.0)
    m.rho = np.zeros_like(m.rho)
    D = 3.0e20
    g = gpu_context(m, "fp64", views=np.array([[45.0, 0.0]]), img_idx=np.array([3]), distance=D)
    st = g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", n_total=m.n_packets,
                       sed_theta_bins=10)
    assert st["escaped"] == m.n_packets and st["scatters"] + st["absorptions"] == 0
    f, c = g.sed()
    nu, w = orc.freq_grid(m.lam_um)
    lnu = np.array([orc.planck(x, float(m.src_tbb[0])) for x in nu])
    lnu *= float(m.src_lum[0]) / np.sum(w * lnu)
    expect = np.broadcast_to(lnu / (4.0 * np.pi * D * D), f.shape)
    ok = c > 300
    assert ok.sum() >= 40
    rel = f[ok] / expect[ok] - 1.0
    assert np.all(np.abs(rel) < 5.0 / np.sqrt(c[ok].astype(float)))
    # the counts themselves: the source spectrum's share per bin (chi^2)
    pj = w * lnu / np.sum(w * lnu)
    exp_c = m.n_packets / 10.0 * pj
    sel = exp_c > 50
    chi = np.sum((c[:, sel] - exp_c[sel]) ** 2 / exp_c[sel]) / (10 * sel.sum())
    assert chi < 1.0 + 4.0 * np.sqrt(2.0 / (10 * sel.sum()))
