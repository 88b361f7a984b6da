"""Helpers that set up the oracle and the HIP library on the same seeded
inputs and compare their outputs (GPU tests only call the HIP path through
the C ABI binding)."""
import numpy as np


def gpu_context(mi, precision="fp64", views=None, img_idx=None, distance=1.0):
    import paper_1203_2941_amd as mc
    ctx = mc.Context(0, precision)
    ctx.from_inputs(mi, views=views, img_idx=img_idx, distance=distance)
    return ctx


def compare_records(rg, ro, tol=1e-6, scale=1.0, allow_frac=1e-6, pos_tol=None):
    """Per-packet parity: same status, wavelength and event counts; escape
    point (within pos_tol, default tol, of `scale`) and direction within tol.
    Packets whose closest decision lies within 1e-9 of a tie on either side
    may legitimately differ; they must be rarer than allow_frac (at least one
    allowed when N is small)."""
    assert len(rg) == len(ro)
    assert np.array_equal(rg["pid"], ro["pid"])
    same = ((rg["status"] == ro["status"]) & (rg["j"] == ro["j"])
            & (rg["n_cross"] == ro["n_cross"]) & (rg["n_scat"] == ro["n_scat"])
            & (rg["n_abs"] == ro["n_abs"]) & (rg["n_mrw"] == ro["n_mrw"])
            & (rg["n_lucy"] == ro["n_lucy"]))
    dp = np.linalg.norm(rg["pos"] - ro["pos"], axis=1) / scale
    dd = np.linalg.norm(rg["dir"] - ro["dir"], axis=1)
    dw = np.abs(rg["weight"] - ro["weight"]) / np.abs(ro["weight"])
    same &= (dp <= (tol if pos_tol is None else pos_tol)) & (dd <= tol) & (dw <= tol)
    near = np.minimum(rg["min_margin"], ro["min_margin"]) < 1e-9
    bad = ~same & ~near
    diverged = ~same & near
    info = {"n": len(rg), "mismatch": int((~same).sum()), "near_tie_diverged": int(diverged.sum()),
            "max_dpos": float(dp[same].max()) if same.any() else 0.0,
            "max_ddir": float(dd[same].max()) if same.any() else 0.0}
    assert not bad.any(), f"packets differ away from ties: {np.flatnonzero(bad)[:10]} {info}"
    assert diverged.sum() <= max(1, int(allow_frac * len(rg))), info
    return info
