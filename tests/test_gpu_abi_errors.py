"""Error paths of the C ABI on a real device: each rejected argument returns
its status and a message, leaves the context usable, and a run after the
failure still matches a clean context bit for bit."""
import ctypes as C

import numpy as np
import pytest

import mcrt_inputs as mi
from tests.pairing import gpu_context

pytestmark = pytest.mark.gpu


def lib():
    from paper_1203_2941_amd import _lib
    return _lib


def dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def status_and_msg(ctx, st):
    L = lib()
    msg = L.lib().mcrt_last_error(ctx.h)
    return st, (msg.decode() if msg else "")


def fresh(precision="fp64"):
    import paper_1203_2941_amd as mc
    return mc.Context(0, precision)


def test_grid_rejects_bad_density():
    L = lib()
    g = fresh()
    org = np.zeros(3)
    for bad in (np.nan, -1e-20, np.inf):
        rho = np.full((4, 4, 4), 1e-18)
        rho[1, 2, 3] = bad
        st = g.lib.mcrt_set_grid(g.h, 4, 4, 4, dp(org), 1.0, C.c_void_p(rho.ctypes.data),
                                 L.FP64, L.HOST)
        st, msg = status_and_msg(g, st)
        assert st == L.EINVAL and "rho" in msg, (bad, msg)
    rho = np.full((4, 4, 4), 1e-18)
    for (nx, dc) in ((0, 1.0), (4, 0.0), (4, np.nan)):
        st = g.lib.mcrt_set_grid(g.h, nx, 4, 4, dp(org), dc, C.c_void_p(rho.ctypes.data),
                                 L.FP64, L.HOST)
        assert st == L.EINVAL
    # queued packets keep their cell in 18 bits per axis
    line = np.full(1 << 18, 1e-18)
    for nx in ((1 << 18) - 1, 1 << 18):
        st = g.lib.mcrt_set_grid(g.h, nx, 1, 1, dp(org), 1.0, C.c_void_p(line.ctypes.data),
                                 L.FP64, L.HOST)
        st, msg = status_and_msg(g, st)
        if nx < (1 << 18):
            assert st == L.OK, msg
        else:
            assert st == L.EINVAL and "per axis" in msg, msg


def test_dust_rejects_bad_tables():
    L = lib()
    m = mi.cube(n=4, n_packets=10)
    g = fresh()
    g.set_grid(m.rho, m.origin, m.dcell)
    lam, fr = m.lam_um.copy(), m.mass_frac.copy()
    ka, ks, gg = m.kabs.copy(), m.ksca.copy(), m.g.copy()

    def call(lam=lam, ka=ka, ks=ks, gg=gg):
        st = g.lib.mcrt_set_dust(g.h, lam.size, dp(lam), fr.size, dp(fr), dp(ka), dp(ks), dp(gg),
                                 -1, 0, None, None)
        return status_and_msg(g, st)

    bad = lam.copy(); bad[5] = bad[4]
    assert call(lam=bad)[0] == L.EINVAL and "increasing" in call(lam=bad)[1]
    bad = lam.copy(); bad[3] = -1.0
    assert call(lam=bad)[0] == L.EINVAL
    bad = ka.copy(); bad[0, 2] = -1.0
    assert call(ka=bad)[0] == L.EINVAL and "kappa" in call(ka=bad)[1]
    bad = ks.copy(); bad[0, 7] = np.nan
    assert call(ks=bad)[0] == L.EINVAL
    for gv in (1.0, -1.0, 1.5):
        bad = gg.copy(); bad[0, 1] = gv
        st, msg = call(gg=bad)
        assert st == L.EINVAL and "|g|" in msg
    assert call()[0] == L.OK


def test_sources_outside_the_grid_and_out_of_order_calls():
    L = lib()
    m = mi.cube(n=4, n_packets=10)
    g = fresh()
    opts = L.RunOpts()
    opts.mode, opts.sed_theta_bins, opts.n_total = L.BW_TICKET, 10, 10
    st = g.lib.mcrt_run_packets(g.h, 0, 10, 0, C.byref(opts), None, None)
    assert status_and_msg(g, st)[0] == L.ESTATE
    pos = np.zeros((1, 3))
    lum = np.array([mi.LSUN])
    tbb = np.array([5800.0])
    st = g.lib.mcrt_set_sources(g.h, 1, dp(pos), dp(lum), None, dp(tbb))
    assert st == L.ESTATE  # before dust and grid
    g.set_grid(m.rho, m.origin, m.dcell)
    g.set_dust(m.lam_um, m.mass_frac, m.kabs, m.ksca, m.g)
    st = g.lib.mcrt_run_packets(g.h, 0, 10, 0, C.byref(opts), None, None)
    assert st == L.ESTATE  # sources missing
    out = np.array([[0.0, 0.0, 2.0 * m.origin[0]]])
    st = g.lib.mcrt_set_sources(g.h, 1, dp(out), dp(lum), None, dp(tbb))
    st, msg = status_and_msg(g, st)
    assert st == L.EINVAL and "outside" in msg
    st = g.lib.mcrt_set_sources(g.h, 1, dp(pos), dp(np.array([-1.0])), None, dp(tbb))
    assert st == L.EINVAL
    # raytracing before views
    img = np.zeros(16)
    st = g.lib.mcrt_set_sources(g.h, 1, dp(pos), dp(lum), None, dp(tbb))
    assert st == L.OK
    st = g.lib.mcrt_raytrace_image(g.h, 4, 4, None, C.c_void_p(img.ctypes.data), None, L.HOST,
                                   None)
    assert st == L.ESTATE


def test_bad_run_options():
    L = lib()
    m = mi.cube(n=4, n_packets=100)
    g = gpu_context(m)
    base = dict(mode="bw_epoch", n_total=100)
    for bad in (dict(epoch_packets=0), dict(sed_theta_bins=0), dict(queue_depth=10),
                dict(blocks_per_cu=33), dict(mrw_tau=5.0, mrw_gamma=0.0),
                dict(mode="frozen", n_iter=0), dict(lucy_tau=float("nan"))):
        kw = dict(base, **bad)
        with pytest.raises(L.McrtError) as e:
            g.run_packets(0, 100, 0, **kw)
        assert e.value.status == L.EINVAL, bad
    with pytest.raises(L.McrtError) as e:
        g.run_packets((1 << 48) - 10, 100, 0, **base)
    assert e.value.status == L.EINVAL


def test_out_of_memory_is_reported_and_recoverable():
    """A record buffer for 2^40 packets (132 TB) cannot be allocated: ENOMEM,
    and the context (and the HIP runtime's error state) stay usable: a
    following run equals the same run on a fresh context."""
    L = lib()
    m = mi.cube(n=8, n_packets=5000, tau_v=2.0, seed=3)
    g = gpu_context(m)
    with pytest.raises(L.McrtError) as e:
        g.run_packets(0, 1 << 40, 0, mode="bw_epoch", record=True, n_total=1 << 40)
    assert e.value.status == L.ENOMEM
    g.reset()
    g.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=512,
                  n_total=m.n_packets)
    h = gpu_context(m)
    h.run_packets(0, m.n_packets, m.seed, mode="bw_epoch", epoch_packets=512,
                  n_total=m.n_packets)
    assert np.array_equal(g.tallies()[0], h.tallies()[0])
    assert np.array_equal(g.sed()[1], h.sed()[1])
