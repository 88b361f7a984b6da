"""The iterative scheme (Eqs. 4-5, repeated passes) and Bjorkman & Wood
re-emission (Eq. 10) reach the same temperatures (sect. 3.3, 3.6)."""
import numpy as np
import pytest

import mcrt_inputs as mi


def test_frozen_iterations_match_serial_bw(orc):
    n = 8
    m = mi.cube(n=n, n_packets=60000, tau_v=4.0)
    it = orc.Oracle(m)
    it.init_T()
    assert np.all(it.T[0] > 0)
    it.run(mode=orc.FROZEN, n_iter=4)
    bw = orc.Oracle(m).run(mode=orc.BW_EPOCH, epoch=1)
    Tb = bw.finalize()[0]
    Ti = it.T[0]
    k = bw.k[0]
    sel = k > 150  # cells with enough absorptions for a per-cent comparison
    assert sel.sum() > 40
    ratio = Ti[sel] / Tb[sel]
    assert np.median(ratio) == pytest.approx(1.0, abs=0.01)
    # MC scatter: T ~ E^(1/5.5), relative E noise ~ 1/sqrt(k) in each run
    z = (ratio - 1.0) / (np.sqrt(2.0 / k[sel]) / 5.5)
    assert np.mean(np.abs(z) < 4) > 0.97


def test_epoch_length_bias_is_small(orc):
    """Longer epochs lag the temperature update; at P = N/25 the global
    energy split between escape bins stays within noise of serial B&W."""
    m = mi.cube(n=12, n_packets=20000, tau_v=4.0)
    a = orc.Oracle(m).run(mode=orc.BW_EPOCH, epoch=1)
    b = orc.Oracle(m).run(mode=orc.BW_EPOCH, epoch=800)
    sa, sb = a.sed.sum(0).astype(float), b.sed.sum(0).astype(float)
    ok = (sa + sb) > 200
    chi = np.sum((sa[ok] - sb[ok]) ** 2 / (sa[ok] + sb[ok]))
    assert chi / ok.sum() < 3.0
