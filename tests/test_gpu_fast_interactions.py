"""The fast interaction kernel of the FP32 walk in immediate B&W (no packet
records) and its slow list, against the oracle's serial B&W at an
independent seed.

- A plain cube: nearly every interaction stays in the fast kernel.
- The same cube at 1e-10 of the luminosity: one packet's energy lies below
  the lower end (3 K) of the Eq. 4 table in every cell, so every absorption
  leaves the fast kernel untouched and the slow kernel takes it whole (the
  FP64 Newton solve of Eq. 4); cell temperatures end between 2 and 8 K.

Temperature z-scores come from the absorption counts (T ~ E^(1/(4+beta)),
beta ~ 1.5); SED counts are compared by chi^2 between two Poisson samples."""
import numpy as np
import pytest

import mcrt_inputs as mi
from tests.pairing import gpu_context

pytestmark = pytest.mark.gpu


def compare_with_serial_bw(orc, m):
    o = orc.Oracle(m).run(mode=orc.BW_EPOCH, epoch=1, seed=m.seed + 777)
    g = gpu_context(m, "fp32")
    st = g.run_packets(0, m.n_packets, m.seed, mode="bw_ticket", n_total=m.n_packets)
    assert st["escaped"] == m.n_packets and st["killed"] == 0
    To, T = o.finalize()[0], g.temperatures()[0]
    k, kg = o.k[0].astype(float), g.tallies()[0][0].astype(float)
    sel = (k > 100) & (kg > 100)
    assert sel.sum() > 50
    z = (T[sel] / To[sel] - 1) / (np.sqrt(1 / k[sel] + 1 / kg[sel]) / 5.5)
    assert np.mean(np.abs(z) < 4) > 0.97, np.mean(np.abs(z) < 4)
    assert abs(np.median(z)) < 0.5, np.median(z)
    so, sg = o.sed.astype(float), g.sed()[1].astype(float)
    ok = (so + sg) > 50
    dof = int(ok.sum())
    c2 = np.sum((so[ok] - sg[ok]) ** 2 / (so[ok] + sg[ok])) / dof
    assert dof > 20 and c2 < 1.0 + 4.0 * np.sqrt(2.0 / dof), (c2, dof)
    # absorptions per packet (binomial-like totals)
    a, b = k.sum(), kg.sum()
    assert abs(b - a) < 4.5 * np.sqrt(a + b), (a, b)
    return To, T


def test_fast_kernel_cube_against_serial_bw(orc):
    m = mi.cube(n=8, n_packets=100_000, tau_v=3.0)
    compare_with_serial_bw(orc, m)


def test_slow_list_takes_interactions_below_the_table(orc):
    m = mi.cube(n=8, n_packets=100_000, tau_v=3.0)
    m.src_lum = m.src_lum * 1e-10
    To, _ = compare_with_serial_bw(orc, m)
    o = orc.Oracle(m)
    xi = float(m.src_lum.sum()) / m.n_packets
    rmin = xi / (4 * np.pi * m.mass_frac[0] * float(np.max(m.rho)) * m.dcell**3)
    # one packet's energy heats no cell to the table's 3 K: all deferred
    assert o.invert_T(0, rmin) < 3.0
    hot = To[To > 0]
    assert 1.5 < np.median(hot) < 10.0


def test_fp32_diffusion_steps_thick_cube(orc):
    """Diffusion steps in the FP32 walk (fast kernel, slow list and per-cell
    flags in immediate B&W; the general kernel in epoch B&W with one packet
    per epoch) on a tau_V = 1e4 cube against the oracle's serial B&W at an
    independent seed: every packet escapes (an interaction cap far above the
    oracle's longest chain bounds the run), the number of diffusion steps and
    the absorbed energy agree within 15 % (full chains amplify last-bit
    differences, so only totals are compared), and the escape SED within its
    Poisson spread."""
    m = mi.cube(n=8, n_packets=2000, tau_v=1e4, nl=20)
    o = orc.Oracle(m).run(mode=orc.BW_EPOCH, epoch=1, mrw_tau=8.0, mrw_gamma=2.0,
                          seed=m.seed + 777)
    assert o.stats["mrw_steps"] > 50 * m.n_packets
    xi = float(m.src_lum.sum()) / m.n_packets
    eo = o.k[0].sum() * xi + o.epath[0].sum()
    so = o.sed.astype(float)
    for mode, kw in (("bw_ticket", {}), ("bw_epoch", {"epoch_packets": 1})):
        print("fp32 diffusion steps,", mode, flush=True)
        g = gpu_context(m, "fp32")
        st = g.run_packets(0, m.n_packets, m.seed, mode=mode, mrw_tau=8.0, mrw_gamma=2.0,
                           n_total=m.n_packets, max_interactions=200_000, **kw)
        assert st["killed"] == 0 and st["escaped"] == m.n_packets, (mode, st)
        assert st["mrw_steps"] == pytest.approx(o.stats["mrw_steps"], rel=0.15), mode
        k, ep, _ = g.tallies()
        eg = k[0].astype(float).sum() * xi + ep[0].sum()
        assert eg == pytest.approx(eo, rel=0.15), mode
        sg = g.sed()[1].astype(float)
        ok = (so + sg) > 30
        dof = int(ok.sum())
        c2 = np.sum((so[ok] - sg[ok]) ** 2 / (so[ok] + sg[ok])) / dof
        assert dof > 10 and c2 < 1.0 + 4.0 * np.sqrt(2.0 / dof), (mode, c2, dof)
