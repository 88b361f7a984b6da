"""Batched persistent launch (one HIP graph over many uneven models)
against per-model launches, and the launch-shape autotuner."""
import numpy as np
import pytest

import mcrt_inputs as mi
from tests.pairing import gpu_context

pytestmark = pytest.mark.gpu


def models():
    specs = [dict(n=24, n_clumps=60, nl=40), dict(n=32, n_clumps=200, nl=64),
             dict(n=16, n_clumps=20, nl=100)]
    return [mi.torus(n_packets=20000 + 5000 * i, seed=i, geo_seed=100 + i, **s)
            for i, s in enumerate(specs)]


def test_batch_equals_individual_runs():
    """FROZEN single pass with the thin-limit temperatures: integer tallies
    are order independent, so the batched graph must reproduce every
    model's per-model launch exactly; repeated graph launches with eager
    work in between give the same result each time."""
    import paper_1203_2941_amd as mc
    ms = models()
    ref = []
    for i, m in enumerate(ms):
        g = gpu_context(m)
        g.init_temperatures()
        g.run_packets(0, m.n_packets, m.seed, mode="frozen", n_iter=1, n_total=m.n_packets)
        ref.append((g.tallies(), g.sed()[1], g.temperatures()))
    ctxs = [gpu_context(m) for m in ms]
    for c in ctxs:
        c.init_temperatures()
    for rep in range(3):
        # the frozen pass overwrites T with its Eq. 4 result: restore the guess
        for c in ctxs:
            c.init_temperatures()
        st = mc.run_batch(ctxs, [m.n_packets for m in ms], [m.seed for m in ms],
                          mode="frozen", n_iter=1)
        for i, (c, m) in enumerate(zip(ctxs, ms)):
            (k, ep, kp), sed, T = ref[i]
            k2, ep2, kp2 = c.tallies()
            assert np.array_equal(k, k2), (rep, i)
            assert np.array_equal(kp, kp2), (rep, i)
            np.testing.assert_allclose(ep2, ep, rtol=1e-10, atol=0)
            assert np.array_equal(c.sed()[1], sed)
            assert st[i]["packets"] == m.n_packets
            # Eq. 4 runs inside the graph: same temperatures as the eager path
            np.testing.assert_allclose(c.current_temperatures(), T, rtol=1e-12, atol=0)
        # eager work between graph launches
        gpu_context(ms[0]).run_packets(0, 1000, 7, mode="bw_ticket", n_total=1000)


def test_batch_ticket_conserves_packets():
    import paper_1203_2941_amd as mc
    ms = models()
    ctxs = [gpu_context(m, "fp32") for m in ms]
    st = mc.run_batch(ctxs, [m.n_packets for m in ms], [m.seed for m in ms], mode="bw_ticket",
                      mrw_tau=50.0)
    for s, m, c in zip(st, ms, ctxs):
        assert s["escaped"] + s["killed"] + s["pah_stopped"] == m.n_packets
        assert int(c.sed()[1].sum()) == s["escaped"]
        T = c.current_temperatures()
        assert np.all(np.isfinite(T)) and T.max() > 0


def test_autotuner_picks_a_candidate(tmp_path, monkeypatch):
    from paper_1203_2941_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    ms = models()
    ctxs = [gpu_context(m, "fp32") for m in ms]
    res = autotune.tune(ctxs, [m.n_packets for m in ms], [m.seed for m in ms],
                        candidates=[(1 << 16, 4, 2), (1 << 18, 3, 2)], mode="bw_ticket")
    assert (res["queue_depth"], res["walk_blocks_per_cu"], res["blocks_per_cu"]) in [
        (1 << 16, 4, 2), (1 << 18, 3, 2)]
    assert res["packets_per_s"] > 0
    again = autotune.tune(ctxs, [m.n_packets for m in ms], [m.seed for m in ms], mode="bw_ticket")
    assert again == res  # served from the cache


def test_batch_against_oracle(orc):
    """A batch of two tori and a refined cube (the leaf walk then serves
    every model), single FROZEN pass from the thin-limit temperatures,
    against the oracle per model: absorption, PAH and SED counts agree up to
    packets that sit within 1e-9 of a decision tie (a handful at most)."""
    import paper_1203_2941_amd as mc
    from tests.test_oracle_refinement import refined_cube
    rc = refined_cube(n=(6, 5, 7), seed=31, frac=0.4, rmax=3, tau=2.0)
    rc.n_packets = 15000
    ms = models()[:2] + [rc]
    ctxs = [gpu_context(m) for m in ms]
    for c in ctxs:
        c.init_temperatures()
    st = mc.run_batch(ctxs, [m.n_packets for m in ms], [m.seed for m in ms], mode="frozen",
                      n_iter=1)
    for c, m, s in zip(ctxs, ms, st):
        o = orc.Oracle(m)
        o.init_T()
        o.run(mode=orc.FROZEN, n_iter=1, n_total=m.n_packets)
        k, ep, kp = c.tallies()
        assert s["packets"] == m.n_packets
        assert np.abs(k.astype(np.int64) - o.k.astype(np.int64)).sum() <= 4
        assert np.abs(kp.astype(np.int64) - o.kpah.astype(np.int64)).sum() <= 4
        assert np.abs(c.sed()[1].astype(np.int64) - o.sed.astype(np.int64)).sum() <= 4
        assert abs(s["crossings"] - o.stats["crossings"]) <= 1e-5 * o.stats["crossings"]
