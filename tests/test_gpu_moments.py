"""GPU (through the C ABI) against the FP64 oracle: scattering events kept
as spherical-harmonic moments and scattered light formed toward views set
after the run (sect. 4), and the g-factor approximation. FP64: per-packet
parity, moments per cell within 1e-10 relative, images within 1e-9; FP32:
moments' totals and images within the FP32 walk's statistical agreement."""
import math

import numpy as np
import pytest

import mcrt_inputs as mi
from tests.pairing import compare_records, gpu_context
from tests.test_gpu_transport import check_cells

pytestmark = pytest.mark.gpu
D = 15.0 * mi.MPC_CM


def kvec(th, ph):
    t, p = math.radians(th), math.radians(ph)
    return [math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)]


def test_moments_fp64_per_cell(orc):
    """Torus with two grain species (different g per wavelength), moments to
    degree 6 at 4 imaged wavelengths, views set before the run: per-packet
    parity, moments per cell, and the peel-off sums."""
    m = mi.torus(n=16, n_clumps=30, n_packets=20000, nl=30, geo_seed=6)
    views, idx = mi.image_views(n_views=3, n_img=4, nl=m.nl)
    o = orc.Oracle(m, views=views, img_idx=idx, distance=D)
    o.run(mode=orc.BW_EPOCH, epoch=4096, record=True, sh_order=7)
    g = gpu_context(m, "fp64", views=views, img_idx=idx, distance=D)
    g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=4096, record=True,
                  n_total=m.n_packets, sh_order=7)
    compare_records(g.records(m.n_packets), o.records, scale=-m.origin[0])
    check_cells(o, g)
    sh = g.scattering_moments()
    assert sh.shape == o.sh.shape and np.abs(o.sh).max() > 0
    np.testing.assert_allclose(sh, o.sh, rtol=1e-10, atol=1e-12 * np.abs(o.sh).max())
    ss = g.scattering()
    np.testing.assert_allclose(ss, o.ssca, rtol=1e-10, atol=1e-12 * np.abs(o.ssca).max())


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_images_toward_views_set_after_the_run(orc, precision):
    """Moments kept by the run, then new views (other angles, same imaged
    wavelengths): the ray-tracer's scattered light comes from the moments
    evaluated toward each new view. The oracle forms the same sums from its
    moments and ray-traces them."""
    m = mi.torus(n=14, n_clumps=25, n_packets=15000, nl=30, geo_seed=7)
    views0, idx = mi.image_views(n_views=2, n_img=5, nl=m.nl)
    order = 6
    o = orc.Oracle(m, views=views0, img_idx=idx, distance=D)
    o.run(mode=orc.BW_EPOCH, epoch=4096, sh_order=order)
    T = o.finalize()
    g = gpu_context(m, precision, views=views0, img_idx=idx, distance=D)
    g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=4096,
                  n_total=m.n_packets, sh_order=order)
    g.set_temperatures(T)
    views = np.array([[17.0, 33.0], [64.0, 250.0], [151.0, -80.0]])
    g.set_views(views, idx, D)
    g.set_scattered_light("moments")
    img_g, sed_g = g.raytrace(20, 18)
    o2 = orc.Oracle(m, views=views, img_idx=idx, distance=D)
    sh = o.sh if precision == "fp64" else g.scattering_moments()
    ss = np.stack([o.sh_view_sums(kvec(*v), sh=sh) for v in views])
    img_o, sed_o = o2.raytrace(20, 18, T=T, ssca=ss)
    if precision == "fp64":
        np.testing.assert_allclose(img_g, img_o, rtol=1e-9, atol=1e-13 * np.abs(img_o).max())
        np.testing.assert_allclose(sed_g, sed_o, rtol=1e-9)
    else:
        for v in range(3):
            for q in range(len(idx)):
                a, b = img_g[v, q].astype(np.float64), img_o[v, q]
                assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b)
    # scattered light differs between views (it is not the peel-off of the run)
    assert np.linalg.norm(img_g[0] - img_g[2]) > 1e-3 * np.linalg.norm(img_g[0])


def test_gfactor_fp64_per_packet(orc):
    """g-factor approximation in the transport: per-packet parity with the
    oracle under the same law."""
    m = mi.torus(n=16, n_clumps=30, n_packets=20000, nl=30, geo_seed=8)
    o = orc.Oracle(m, scat_law=orc.SCAT_GFACTOR)
    o.run(mode=orc.BW_EPOCH, epoch=4096, record=True)
    g = gpu_context(m, "fp64")
    g.set_scattering_law("gfactor")
    g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=4096, record=True,
                  n_total=m.n_packets)
    compare_records(g.records(m.n_packets), o.records, scale=-m.origin[0])
    check_cells(o, g)
    # and back to Henyey-Greenstein
    g.set_scattering_law("hg")
    o2 = orc.Oracle(m).run(mode=orc.BW_EPOCH, epoch=4096, record=True)
    g.reset()
    g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=4096, record=True,
                  n_total=m.n_packets)
    compare_records(g.records(m.n_packets), o2.records, scale=-m.origin[0])


def test_moment_errors():
    import paper_1203_2941_amd as mc
    m = mi.cube(n=8, n_packets=100, tau_v=1.0)
    g = gpu_context(m)
    assert g.scattering_moments() is None
    with pytest.raises(mc.McrtError, match="status -1"):
        g.run_packets(0, 100, 0, mode="bw_epoch", sh_order=10)
    with pytest.raises(mc.McrtError, match="status -1"):
        g.set_scattered_light(5)
    with pytest.raises(mc.McrtError, match="status -1"):
        g.set_scattering_law(3)
