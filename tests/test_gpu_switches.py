"""GPU (through the C ABI) against the FP64 oracle for the paper-literal
switches: a new optical-depth draw per cell (footnote to the sect. 2
interaction test), m equal-energy source strata (Eq. 1), and the printed
ray-tracer form (Eqs. 13-14). FP64: per-packet parity as for the default
transport (events exact, end point and direction within 1e-6), images and
gradients within 1e-10; FP32: images within 1e-5 relative L2, per-packet
first flights."""
import numpy as np
import pytest

import mcrt_inputs as mi
from tests.pairing import compare_records, gpu_context
from tests.test_gpu_transport import check_cells

pytestmark = pytest.mark.gpu
D = 15.0 * mi.MPC_CM


@pytest.mark.parametrize("mode", ["bw_epoch", "frozen"])
def test_per_cell_draws_fp64_per_packet(orc, mode):
    """Clumpy 24^3 torus (empty, thin and thick cells) with scattering,
    absorption and re-emission; every cell entered takes its own draw."""
    m = mi.torus(n=24, n_clumps=60, n_packets=20000, nl=30, geo_seed=2)
    o = orc.Oracle(m)
    g = gpu_context(m)
    if mode == "frozen":
        o.init_T()
        g.init_temperatures()
        o.run(record=True, mode=orc.FROZEN, n_iter=1, tau_mode=orc.TAU_PER_CELL)
        st = g.run_packets(0, m.n_packets, m.seed, mode="frozen", n_iter=1, record=True,
                           n_total=m.n_packets, tau_mode="per_cell")
    else:
        o.run(record=True, mode=orc.BW_EPOCH, epoch=2048, tau_mode=orc.TAU_PER_CELL)
        st = g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=2048,
                           record=True, n_total=m.n_packets, tau_mode="per_cell")
    info = compare_records(g.records(m.n_packets), o.records, tol=1e-6, scale=-m.origin[0])
    print(mode, info, flush=True)
    check_cells(o, g)
    for key in ("escaped", "scatters", "absorptions", "crossings", "lucy_deposits"):
        assert st[key] == o.stats[key], key


def test_per_cell_draws_fp32_first_flight(orc):
    """FP32 walk with per-cell draws: packets that leave without an
    interaction keep their direction and wavelength, and their number of
    crossings matches the oracle's (same draws, cell by cell)."""
    m = mi.cube(n=16, n_packets=30000, tau_v=0.7, seed=9)
    o = orc.Oracle(m).run(record=True, mode=orc.BW_EPOCH, epoch=4096, lucy_tau=0.0,
                          tau_mode=orc.TAU_PER_CELL)
    g = gpu_context(m, "fp32")
    g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=4096, record=True,
                  lucy_tau=0.0, n_total=m.n_packets, tau_mode="per_cell")
    rg, ro = g.records(m.n_packets), o.records
    direct = (ro["n_scat"] + ro["n_abs"] + ro["n_mrw"] == 0) & (ro["status"] == orc.ESCAPED)
    gd = (rg["n_scat"] + rg["n_abs"] + rg["n_mrw"] == 0) & (rg["status"] == orc.ESCAPED)
    both = direct & gd
    assert both.sum() > 0.95 * direct.sum() and direct.sum() > 0.3 * m.n_packets
    np.testing.assert_allclose(rg["dir"][both], ro["dir"][both], atol=2e-6)
    assert np.array_equal(rg["j"][both], ro["j"][both])
    assert np.mean(rg["n_cross"][both] == ro["n_cross"][both]) > 0.999


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_source_strata_per_packet(orc, precision):
    """Stratified source wavelengths: the same bin per packet (the draw is
    made in FP64 in both precisions); FP64 runs the whole history."""
    m = mi.cube(n=16, n_packets=12000, tau_v=1.0, seed=10)
    strata = 97
    o = orc.Oracle(m).run(record=True, mode=orc.BW_EPOCH, epoch=4096, src_strata=strata)
    g = gpu_context(m, precision)
    g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=4096, record=True,
                  n_total=m.n_packets, src_strata=strata)
    rg = g.records(m.n_packets)
    if precision == "fp64":
        compare_records(rg, o.records, tol=1e-6, scale=-m.origin[0])
        check_cells(o, g)
    else:
        # the first wavelength is that of the emission; compare packets that
        # escape without an interaction
        ro = o.records
        direct = (ro["n_scat"] + ro["n_abs"] == 0) & (rg["n_scat"] + rg["n_abs"] == 0)
        assert direct.sum() > 1000
        assert np.array_equal(rg["j"][direct], ro["j"][direct])


def rt_setup(orc, precision, nimg, npx=24, npy=20):
    m = mi.torus(n=20, n_clumps=80, n_packets=10, nl=30, geo_seed=3)
    views, idx = mi.image_views(n_views=3, n_img=nimg, nl=m.nl)
    views[1, 1] = 37.0
    rng = np.random.default_rng(4)
    nc = m.nx * m.ny * m.nz
    T = rng.uniform(80.0, 1500.0, (m.ns, nc))
    T[m.pah_species] = 0.0
    ssca = rng.uniform(0.0, 1.0, (3, nimg, nc)) * 1e40
    o = orc.Oracle(m, views=views, img_idx=idx, distance=D)
    g = gpu_context(m, precision, views=views, img_idx=idx, distance=D)
    g.set_temperatures(T)
    g.set_scattering(ssca)
    g.set_raytrace_mode("abs_literal")
    return m, o, g, T, ssca, npx, npy


@pytest.mark.parametrize("nimg", [5, 16])
def test_literal_images_and_gradient_fp64(orc, nimg):
    m, o, g, T, ssca, npx, npy = rt_setup(orc, "fp64", nimg)
    lit = orc.RT_ABS_LITERAL
    img_o, sed_o = o.raytrace(npx, npy, T=T, ssca=ssca, rt_mode=lit)
    img_g, sed_g = g.raytrace(npx, npy)
    np.testing.assert_allclose(img_g, img_o, rtol=1e-10, atol=1e-14 * np.abs(img_o).max())
    np.testing.assert_allclose(sed_g, sed_o, rtol=1e-10)
    rng = np.random.default_rng(5)
    w = rng.uniform(0.0, 1.0, img_o.shape)
    gw = rng.normal(size=sed_o.shape)
    d_o = o.raytrace_adjoint(npx, npy, w_img=w, w_sed=gw, T=T, ssca=ssca, rt_mode=lit)
    d_g = g.raytrace_adjoint(npx, npy, w_img=w, w_sed=gw)
    assert np.linalg.norm(d_g - d_o) <= 1e-10 * np.linalg.norm(d_o)


@pytest.mark.parametrize("nimg", [5, 16])
def test_literal_images_fp32(orc, nimg):
    m, o, g, T, ssca, npx, npy = rt_setup(orc, "fp32", nimg, 40, 36)
    lit = orc.RT_ABS_LITERAL
    img_o, _ = o.raytrace(npx, npy, T=T, ssca=ssca, rt_mode=lit)
    img_g, _ = g.raytrace(npx, npy)
    img_g = img_g.astype(np.float64)
    for v in range(img_o.shape[0]):
        for q in range(img_o.shape[1]):
            a, b = img_g[v, q], img_o[v, q]
            assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b)
    rng = np.random.default_rng(6)
    w = rng.uniform(0.0, 1.0, img_o.shape)
    d_o = o.raytrace_adjoint(npx, npy, w_img=w, T=T, ssca=ssca, rt_mode=lit)
    d_g = g.raytrace_adjoint(npx, npy, w_img=w.astype(np.float32))
    assert np.linalg.norm(d_g - d_o) <= 1e-4 * np.linalg.norm(d_o)


def test_raytrace_mode_switch_back():
    """Switching back to the chord form rebuilds the source functions."""
    import paper_1203_2941_amd as mc
    m = mi.torus(n=12, n_clumps=20, n_packets=10, nl=30, geo_seed=4)
    views, idx = mi.image_views(n_views=2, n_img=4, nl=m.nl)
    g = gpu_context(m, "fp64", views=views, img_idx=idx, distance=D)
    rng = np.random.default_rng(7)
    T = rng.uniform(80.0, 1500.0, (m.ns, m.nx * m.ny * m.nz))
    T[m.pah_species] = 0.0
    g.set_temperatures(T)
    a, _ = g.raytrace(10, 10)
    g.set_raytrace_mode("abs_literal")
    b, _ = g.raytrace(10, 10)
    g.set_raytrace_mode("ext")
    c, _ = g.raytrace(10, 10)
    assert np.array_equal(a, c)
    assert np.linalg.norm(a - b) > 1e-3 * np.linalg.norm(a)
    with pytest.raises(mc.McrtError):
        g.set_raytrace_mode(7)


def test_pah_dissociation_fp64_per_packet(orc):
    """PAH photodissociation (Eq. 8) in the second stage: a cooling time that
    makes about half of the PAH packets' cells dissociate; those packets start
    from the source. Per-packet parity of both passes and the same cells."""
    from tests.test_oracle_pah_dissociation import t_star
    m = mi.torus(n=16, n_clumps=30, n_packets=40000, nl=40, geo_seed=5)
    o = orc.Oracle(m)
    o.run(mode=orc.BW_EPOCH, epoch=5000, record=True)
    g = gpu_context(m)
    g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=5000, record=True,
                  n_total=m.n_packets)
    compare_records(g.records(m.n_packets), o.records, scale=-m.origin[0])
    kp = o.kpah.copy()
    busy = np.flatnonzero(kp)
    # a cooling time between two distinct thresholds near the packet-weighted
    # median
    ts = np.array([t_star(o, m, c) for c in busy])
    order = np.argsort(ts)
    cum = np.cumsum(kp[busy][order]) / kp.sum()
    k = min(int(np.searchsorted(cum, 0.5)), len(order) - 2)
    while ts[order[k + 1]] == ts[order[k]] and k + 2 < len(order):
        k += 1
    tc = float(np.sqrt(ts[order[k]] * ts[order[k + 1]]))
    flag = o.pah_dissociates(pah_nc=60.0, pah_tcool=tc)
    assert 0.1 < kp[flag].sum() / kp.sum() < 0.9
    npah = int(kp.sum())
    o.pah_pass(mode=orc.BW_EPOCH, epoch=5000, record=True, pah_nc=60.0, pah_tcool=tc)
    st = g.run_pah(m.seed, mode="bw_epoch", epoch_packets=5000, record=True, pah_nc=60.0,
                   pah_tcool=tc)
    assert st["packets"] == npah
    compare_records(g.records(npah), o.records, scale=-m.origin[0])
    check_cells(o, g)


def test_constant_density_envelope_voxelizer(orc):
    """The envelope of the sect. 3.6 run-time comparison (power 0) on the
    device against the oracle's cell averages."""
    m = mi.replica(n=40, n_packets=10)
    g = gpu_context(m)
    ref = orc.voxelize_shell(m.nx, m.ny, m.nz, m.origin, m.dcell, m.geometry)
    assert np.count_nonzero(ref) > 0.3 * ref.size
    np.testing.assert_allclose(g.density(), ref.ravel(), rtol=1e-12, atol=0)
