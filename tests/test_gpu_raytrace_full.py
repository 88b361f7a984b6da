"""Ray-tracer and adjoint at the benchmark's size: the 256^3 clumpy torus,
8 views x 16 imaged wavelengths, 512^2 pixels (the launch configuration the
benchmark times).

- Forward against the oracle at full grid size on a 16^2 image (the same
  kernels, fewer pixel rays so the oracle finishes in seconds): FP64 within
  1e-10 relative per pixel, FP32 within 1e-5 relative L2 per image (images
  within FP32's range).
- Adjoint (FP64) against central differences of the FP64 forward at 512^2:
  64 sampled cells (32 inside clumps, 32 between them) and 8 random
  directions in density space, relative steps h = 1e-4, each derivative
  within 1e-4 relative (the step's truncation error (h tau)^2/6 stays below
  1e-6 for the optical depths that carry any transmitted light; rays that
  miss the perturbed cells give identical pixels, so nothing cancels).
- FP32 adjoint against FP64 within 1e-4 relative L2.

Temperatures are a seeded smooth field and the scattering sums are zero, so
no transport run is needed for the source functions."""
import numpy as np
import pytest

import mcrt_inputs as mi
from tests.pairing import gpu_context

pytestmark = pytest.mark.gpu
D = 15.0 * mi.MPC_CM
NPIX = 512


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    oracle.build(force=False)
    return oracle


def smooth_T(m):
    """T_s(r) = T0_s (r_in / max(r, r_in))^0.4 at cell centres, seeded +-5 %
    jitter; the PAH species has none."""
    ax = [m.origin[k] + (np.arange(n) + 0.5) * m.dcell for k, n in enumerate((m.nx, m.ny, m.nz))]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    r = np.sqrt(x * x + y * y + z * z).ravel()
    r_in = m.geometry["r_in"]
    base = (r_in / np.maximum(r, r_in)) ** 0.4
    rng = np.random.default_rng(11)
    T = np.zeros((m.ns, r.size))
    for s, t0 in enumerate((1500.0, 1700.0)):
        T[s] = t0 * base * (1.0 + 0.05 * (rng.random(r.size) - 0.5))
    if m.pah_species >= 0:
        T[m.pah_species] = 0.0
    return T


@pytest.fixture(scope="module")
def big():
    print("torus 256^3, 8 views x 16 wavelengths", flush=True)
    m = mi.torus(n=256, n_packets=10)
    views, idx = mi.image_views(n_views=8, n_img=16, nl=m.nl)
    T = smooth_T(m)
    ctx = {}
    for p in ("fp64", "fp32"):
        g = gpu_context(m, p, views=views, img_idx=idx, distance=D)
        g.reset()
        g.set_temperatures(T)
        ctx[p] = g
    return m, views, idx, T, ctx


def test_forward_full_grid_against_oracle(orc, big):
    m, views, idx, T, ctx = big
    o = orc.Oracle(m, views=views, img_idx=idx, distance=D)
    n = 16
    img_o, sed_o = o.raytrace(n, n, T=T)
    assert np.abs(img_o).max() > 0
    img64, sed64 = ctx["fp64"].raytrace(n, n)
    scale = np.abs(img_o).max(axis=(2, 3), keepdims=True)
    np.testing.assert_allclose(img64, img_o, rtol=1e-10, atol=1e-14 * scale.max())
    np.testing.assert_allclose(sed64, sed_o, rtol=1e-10)
    img32, _ = ctx["fp32"].raytrace(n, n)
    img32 = img32.astype(np.float64)
    checked = 0
    for v in range(img_o.shape[0]):
        for q in range(img_o.shape[1]):
            b = img_o[v, q]
            # images whose brightest pixel lies below 1e6 x FP32's smallest
            # normal number (a wavelength seen through the torus' full
            # extinction, down to 1e-126) are not representable in FP32
            if np.abs(b).max() < 1e6 * np.finfo(np.float32).tiny:
                continue
            assert np.linalg.norm(img32[v, q] - b) <= 1e-5 * np.linalg.norm(b), (v, q)
            checked += 1
    assert checked >= 32


def test_adjoint_full_size_sampled_cells_and_directions(big):
    import torch
    m, views, idx, T, ctx = big
    g = ctx["fp64"]
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(5)
    W = torch.tensor(rng.random((len(views), len(idx), NPIX, NPIX)), device=dev)
    grad = g.raytrace_adjoint_device(NPIX, NPIX, w_img=W).cpu().numpy()
    rho_h = g.density()
    rho = torch.tensor(rho_h, device=dev)
    img_p = torch.empty_like(W)
    img_m = torch.empty_like(W)

    def dloss(rp, rm):
        g.raytrace_device(NPIX, NPIX, rho_rt=rp, img=img_p)
        g.raytrace_device(NPIX, NPIX, rho_rt=rm, img=img_m)
        # pixels whose rays miss the change are identical in both images
        return float((W * (img_p - img_m)).sum())

    # sensitivities rho_c dL/drho_c; cells picked among those carrying light
    sens = np.abs(grad * rho_h)
    clump = rho_h > 10.0 * m.geometry["rho_inter"]
    inter = (rho_h > 0) & ~clump
    picks = []
    for sel in (clump, inter):
        cand = np.flatnonzero(sel & (sens >= 1e-3 * sens[sel].max()))
        assert cand.size >= 32
        picks += list(rng.choice(cand, size=32, replace=False))
    print(f"FD over {len(picks)} cells", flush=True)
    h = 1e-4
    worst = 0.0
    for c in picks:
        rp = rho.clone(); rp[c] *= 1.0 + h
        rm = rho.clone(); rm[c] *= 1.0 - h
        fd = dloss(rp, rm) / (2.0 * h * rho_h[c])
        err = abs(fd - grad[c]) / abs(grad[c])
        worst = max(worst, err)
        assert err <= 1e-4, (int(c), fd, grad[c])
    print(f"cells: worst relative difference {worst:.2e}", flush=True)
    for k in range(8):
        v = torch.tensor(rng.normal(size=rho_h.size), device=dev) * rho
        hd = 1e-4
        fd = dloss(rho + hd * v, rho - hd * v) / (2.0 * hd)
        an = float(np.dot(grad, v.cpu().numpy()))
        assert abs(fd - an) <= 1e-4 * abs(an), (k, fd, an)


def test_fp32_adjoint_against_fp64_full_size(big):
    import torch
    m, views, idx, T, ctx = big
    rng = np.random.default_rng(5)
    Wh = rng.random((len(views), len(idx), NPIX, NPIX))
    g64 = ctx["fp64"].raytrace_adjoint_device(
        NPIX, NPIX, w_img=torch.tensor(Wh, device="cuda")).cpu().numpy()
    g32 = ctx["fp32"].raytrace_adjoint_device(
        NPIX, NPIX, w_img=torch.tensor(Wh.astype(np.float32), device="cuda")).cpu().numpy()
    rel = np.linalg.norm(g32.astype(np.float64) - g64) / np.linalg.norm(g64)
    print(f"FP32 vs FP64 gradient, relative L2 {rel:.2e}", flush=True)
    assert rel <= 1e-4
