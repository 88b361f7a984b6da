"""GPU (HIP, through the C ABI) against the FP64 oracle on the code paths the
benchmark runs: scattering sums accumulated during transport and the images
made from them, several sources, the FP32 walk in immediate B&W without
packet records, FP32 Lucy deposits at packet energies beyond FLT_MAX, and
the MRW shortcuts of the record-free kernels."""
import dataclasses
import math

import time

import numpy as np
import pytest

import mcrt_inputs as mi
from tests.pairing import compare_records, gpu_context

pytestmark = pytest.mark.gpu
D = 15.0 * mi.MPC_CM


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    oracle.build(force=False)
    return oracle


def test_scattering_sums_and_images_fp64(orc):
    """FP64 immediate-epoch run with 8 views and 16 imaged wavelengths: the
    per-packet histories agree, so the HG-weighted scattering sums agree cell
    by cell (sums of the same terms in another order); images made from each
    side's own temperatures and sums agree to rounding."""
    m = mi.torus(n=20, n_clumps=60, n_packets=30000, nl=40, seed=2)
    views, idx = mi.image_views(8, 16, nl=m.nl)
    o = orc.Oracle(m, views=views, img_idx=idx, distance=D)
    o.run(mode=orc.BW_EPOCH, epoch=4096, record=True)
    g = gpu_context(m, "fp64", views=views, img_idx=idx, distance=D)
    g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=4096, record=True,
                  n_total=m.n_packets)
    info = compare_records(g.records(m.n_packets), o.records, scale=-m.origin[0])
    print(info, flush=True)
    sg, so = g.scattering(), o.ssca
    assert so.shape == sg.shape and np.count_nonzero(so) > 1000
    if info["mismatch"] == 0:
        np.testing.assert_allclose(sg, so, rtol=1e-9, atol=1e-13 * so.max())
    else:
        assert np.linalg.norm(sg - so) <= 1e-3 * np.linalg.norm(so)
    To = o.finalize()
    Tg = g.temperatures()
    np.testing.assert_allclose(Tg, To, rtol=1e-4, atol=0)
    npx, npy = 36, 30
    img_o, sed_o = o.raytrace(npx, npy, T=To, ssca=so)
    img_g, sed_g = g.raytrace(npx, npy)
    tol = 1e-8 if info["mismatch"] == 0 else 1e-3
    for v in range(img_o.shape[0]):
        for q in range(img_o.shape[1]):
            a, b = img_g[v, q], img_o[v, q]
            assert np.linalg.norm(a - b) <= tol * np.linalg.norm(b), (v, q)
    np.testing.assert_allclose(sed_g, sed_o, rtol=tol)


def test_two_sources_fp64_per_packet(orc):
    """Source chosen in proportion to its luminosity (two sources, 1:3, at
    different positions and temperatures): per-packet parity."""
    base = mi.cube(n=16, n_packets=20000, tau_v=1.0, seed=4)
    half = -base.origin[0]
    m = dataclasses.replace(base, src_pos=np.array([[-0.3, 0.1, 0.2], [0.25, -0.2, 0.1]]) * half,
                            src_lum=np.array([1.0, 3.0]) * mi.LSUN,
                            src_tbb=np.array([5800.0, 3000.0]))
    o = orc.Oracle(m).run(mode=orc.BW_EPOCH, epoch=2048, record=True)
    g = gpu_context(m)
    st = g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=2048, record=True,
                       n_total=m.n_packets)
    compare_records(g.records(m.n_packets), o.records, scale=half)
    k, ep, _ = g.tallies()
    assert np.array_equal(k, o.k)
    assert np.array_equal(g.sed()[1], o.sed)
    assert st["escaped"] == o.stats["escaped"]


def test_fp32_lucy_with_packet_energy_above_float_max(orc):
    """Thin cube (every cell thin) with packet energy xi = 3.3e39 erg/s, beyond
    the FP32 range: the FP32 walk's Lucy deposits (Eq. 9) must stay finite and
    match the FP64 oracle. Directions of the first flight are the same draws,
    so per-cell energies agree up to the few packets that interact."""
    base = mi.cube(n=16, n_packets=30000, tau_v=1e-3, seed=6)
    m = dataclasses.replace(base, src_lum=np.array([1e44]))
    o = orc.Oracle(m).run(mode=orc.BW_EPOCH, epoch=4096)
    assert o.xi() > 3.4e38
    g = gpu_context(m, "fp32")
    st = g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=4096,
                       n_total=m.n_packets)
    assert st["lucy_deposits"] > 10 * m.n_packets
    _, ep, _ = g.tallies()
    assert np.all(np.isfinite(ep))
    assert ep.sum() == pytest.approx(o.epath.sum(), rel=2e-3)
    big = o.epath > 1e-3 * o.epath.max()
    np.testing.assert_allclose(ep[big], o.epath[big], rtol=3e-2)
    # a single packet of 3.3e39 erg/s absorbed in a cell of this tiny mass puts
    # Eq. 10's temperature (E + xi) above the 1e5 K ceiling in both codes; the
    # few such absorptions are the same packets on both sides
    assert abs(st["clamped_T"] - o.stats["clamped_T"]) <= 2
    # Eq. 4 from the path energies: the cells next to a 1e44 erg/s source sit
    # at the 1e5 K ceiling in both codes; the others agree like the energies
    T = g.temperatures()
    To = o.finalize()
    assert np.all(np.isfinite(T))
    cool = (To < 0.999e5) & big
    assert cool.sum() > 100
    np.testing.assert_allclose(T[cool], To[cool], rtol=1e-2)
    assert abs(int((T >= 0.999e5).sum()) - int((To >= 0.999e5).sum())) <= 2


@pytest.mark.parametrize("precision", [
    "fp64",
    "fp32",
])
def test_mrw_shortcuts_change_nothing(orc, precision):
    """The record-free kernels skip the exact Rosseland mean (and in immediate
    B&W the Eq. 4 inversion) when an upper bound of kappa_R already rules a
    diffusion step out. Runs with and without records must take the same
    steps. One epoch makes every packet independent in BW_EPOCH; in
    immediate B&W one packet per call makes the order deterministic."""
    m = mi.cube(n=8, n_packets=150, tau_v=1e5, nl=12, seed=8)
    t0 = time.time()
    out = []
    for rec in (True, False):
        g = gpu_context(m, precision)
        st = g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=10 ** 9,
                           mrw_tau=8.0, mrw_gamma=2.0, record=rec, n_total=m.n_packets)
        print(f"epoch run, records {rec}: {st['mrw_steps']} diffusion steps, "
              f"{time.time() - t0:.1f} s", flush=True)
        k, ep, _ = g.tallies()
        out.append((st, k, ep, g.sed()[1].copy()))
    (sa, ka, ea, fa), (sb, kb, eb, fb) = out
    assert sa["mrw_steps"] > 1000 and sa["mrw_steps"] == sb["mrw_steps"]
    assert np.array_equal(ka, kb) and np.array_equal(fa, fb)
    np.testing.assert_allclose(ea, eb, rtol=1e-12, atol=0)
    out = []
    # one packet per call runs its chain in a single lane (about 0.15 ms per
    # diffusion step, 2e3 to 7e4 steps per packet here): the first n of
    # n_total packets
    n, n_total = 8, 40
    for rec in (True, False):
        g = gpu_context(m, precision)
        tot = {"mrw_steps": 0, "crossings": 0}
        for i in range(n):
            st = g.run_packets(i, 1, m.seed, mode="bw_ticket", mrw_tau=8.0, mrw_gamma=2.0,
                               record=rec, n_total=n_total)
            for key in tot:
                tot[key] += st[key]
            print(f"one-packet call {i}, records {rec}: {st['mrw_steps']} diffusion steps, "
                  f"{time.time() - t0:.1f} s", flush=True)
        k, ep, _ = g.tallies()
        out.append((tot, k, ep))
    (ta, ka, ea), (tb, kb, eb) = out
    assert ta["mrw_steps"] > 100 and ta == tb
    assert np.array_equal(ka, kb)
    np.testing.assert_allclose(ea, eb, rtol=1e-12, atol=0)


def test_fp32_immediate_bw_torus_against_serial_bw(orc):
    """The benchmark's transport (FP32 walk, immediate B&W, no packet records,
    MRW armed, 8 views x 16 imaged wavelengths, PAH second stage) on a 48^3
    torus against the oracle's serial B&W with an independent seed.

    Both sides run the same number of packets with the same packet energy
    (B&W temperatures depend on xi: (E + xi) in Eq. 10), the GPU in ten
    consecutive calls of one run. Noise is independent on the two sides, so
    the statistics below are calibrated: per-cell temperature z-scores from
    the absorption counts (T ~ E^(1/(4+beta)), beta ~ 1.5), SED and PAH count
    chi^2 between two Poisson samples, binomial escape fractions, crossings
    per packet, and scattering-sum totals per view and wavelength against the
    spread of the ten GPU chunks (which also holds the run's drift, so that
    test is conservative)."""
    nl = 40
    n_o, chunks = 200_000, 10
    n_g = n_o
    n_c = n_o // chunks
    m = mi.torus(n=48, n_clumps=300, n_packets=n_o, nl=nl, seed=11)
    views, idx = mi.image_views(8, 16, nl=nl)
    o = orc.Oracle(m, views=views, img_idx=idx, distance=D)
    o.run(mode=orc.BW_EPOCH, epoch=1, record=True, mrw_tau=50.0)
    cross_o = o.records["n_cross"].astype(np.float64)
    so1 = o.ssca.copy()
    st_o = dict(o.stats)
    kpah_o = o.kpah.astype(np.float64).copy()
    o.pah_pass(mode=orc.BW_EPOCH, epoch=1, mrw_tau=50.0)
    To = o.finalize()
    k_o = o.k.astype(np.float64)

    g = gpu_context(m, "fp32", views=views, img_idx=idx, distance=D)
    seed_g = 987654321
    parts, st_g = [], {"escaped": 0, "pah_stopped": 0, "crossings": 0, "killed": 0}
    prev = np.zeros_like(so1)
    for c in range(chunks):
        st = g.run_packets(c * n_c, n_c, seed_g, mode="bw_ticket", mrw_tau=50.0, n_total=n_g)
        for key in st_g:
            st_g[key] += st[key]
        cur = g.scattering()
        parts.append((cur - prev).sum(axis=2))
        prev = cur
    kpah_g = g.tallies()[2].astype(np.float64)
    assert st_g["killed"] == 0
    g.run_pah(seed_g, mode="bw_ticket", mrw_tau=50.0)
    Tg = g.temperatures()
    k_g = g.tallies()[0].astype(np.float64)

    # escape and PAH-stop fractions (binomial), crossings per packet
    for key in ("escaped", "pah_stopped"):
        p_o, p_g = st_o[key] / n_o, st_g[key] / n_g
        p = (st_o[key] + st_g[key]) / (n_o + n_g)
        z = (p_g - p_o) / math.sqrt(p * (1 - p) * (1 / n_o + 1 / n_g))
        assert abs(z) < 4.5, (key, z)
    sd = cross_o.std()
    z = (st_g["crossings"] / n_g - cross_o.mean()) / (sd * math.sqrt(1 / n_o + 1 / n_g))
    assert abs(z) < 4.5, ("crossings per packet", z)

    def chi2(a, na, b, nb, floor=30):
        ok = (a + b) > floor
        num = (a[ok] / na - b[ok] / nb) ** 2
        den = a[ok] / na ** 2 + b[ok] / nb ** 2
        return float(np.sum(num / den) / ok.sum()), int(ok.sum())

    # chi^2 per degree of freedom within 4 sigma (sqrt(2/dof)) of 1
    c2, dof = chi2(kpah_o, n_o, kpah_g, n_g)
    assert dof > 40 and c2 < 1.0 + 4.0 * math.sqrt(2.0 / dof), ("PAH counts", c2, dof)
    f_o, f_g = o.sed.astype(np.float64), g.sed()[1].astype(np.float64)
    c2, dof = chi2(f_o, n_o, f_g, n_g)
    assert dof > 50 and c2 < 1.0 + 4.0 * math.sqrt(2.0 / dof), ("SED", c2, dof)

    # temperatures of well-sampled cells
    sel = (k_o[:2] > 40) & (k_g[:2] > 40)
    assert sel.sum() > 200
    z = (Tg[:2][sel] / To[:2][sel] - 1.0) / (np.sqrt(1 / k_o[:2][sel] + 1 / k_g[:2][sel]) / 5.5)
    assert np.mean(np.abs(z) < 4) > 0.97, np.mean(np.abs(z) < 4)
    assert abs(np.median(z)) < 0.5, np.median(z)
    # absorbed energy per thermal species, as a fraction of the luminosity
    for s in range(2):
        a, b = k_o[s].sum(), k_g[s].sum()
        zz = (b / n_g - a / n_o) / math.sqrt(a / n_o ** 2 + b / n_g ** 2)
        assert abs(zz) < 4.5, ("absorptions", s, zz)

    # scattering sums per view and imaged wavelength (first stage): totals of
    # the two runs against the chunk spread (variance of a total: chunks x
    # the chunk variance, on each side)
    c = np.asarray(parts)
    sd = c.std(axis=0, ddof=1)
    tot_g, tot_o = c.sum(axis=0), so1.sum(axis=2)
    ok = sd > 0
    z = (tot_g[ok] - tot_o[ok]) / (sd[ok] * math.sqrt(2.0 * chunks))
    assert z.size > 64  # of 8 views x 16 wavelengths; some imaged wavelengths barely scatter
    assert np.mean(z ** 2) < 1.5, np.mean(z ** 2)
    assert np.max(np.abs(z)) < 5.0, np.max(np.abs(z))


def test_interaction_cap_one_and_epoch_of_one_packet(orc):
    """Edge cases of the options: every packet killed at its first
    interaction (cap 1), and B&W epochs of a single packet (serial B&W)."""
    m = mi.cube(n=8, n_packets=4000, tau_v=3.0, seed=9)
    o = orc.Oracle(m).run(mode=orc.BW_EPOCH, epoch=1, record=True, max_int=1)
    g = gpu_context(m)
    st = g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=1, record=True,
                       max_interactions=1, n_total=m.n_packets)
    assert st["killed"] == o.stats["killed"] > 1000
    assert st["escaped"] + st["killed"] == m.n_packets
    compare_records(g.records(m.n_packets), o.records, scale=-m.origin[0])
    m2 = mi.cube(n=8, n_packets=1500, tau_v=2.0, seed=10)
    o2 = orc.Oracle(m2).run(mode=orc.BW_EPOCH, epoch=1, record=True)
    g2 = gpu_context(m2)
    g2.run_packets(0, m2.n_packets, m2.seed, mode="bw_epoch", epoch_packets=1, record=True,
                   n_total=m2.n_packets)
    compare_records(g2.records(m2.n_packets), o2.records, scale=-m2.origin[0])
    k, ep, _ = g2.tallies()
    assert np.array_equal(k, o2.k)
