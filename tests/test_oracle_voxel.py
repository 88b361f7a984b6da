"""Pins of the model voxelizers (clumpy torus of sect. 6, Eq. 21; r^-2 shell)."""
import math

import numpy as np
import pytest

import mcrt_inputs as mi


def test_torus_cells(orc):
    m = mi.torus(n=32, n_clumps=60, n_packets=10)
    geo = m.geometry
    rho = orc.voxelize_torus(m.nx, m.ny, m.nz, m.origin, m.dcell, geo)
    vals = set(np.unique(rho).tolist())
    assert vals <= {0.0, geo["rho_inter"], geo["rho_clump"]}
    ax = m.origin[0] + (np.arange(32) + 0.5) * m.dcell
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    P = np.stack([X, Y, Z], -1)
    d2 = ((P[..., None, :] - geo["centres"][None, None, None]) ** 2).sum(-1).min(-1)
    inclump = d2 <= geo["r_clump"] ** 2
    assert np.array_equal(rho == geo["rho_clump"], inclump)
    r2 = (P**2).sum(-1)
    wedge = (r2 >= geo["r_in"] ** 2) & (r2 <= geo["r_out"] ** 2) & (Z**2 <= r2 * geo["sin_theta1"] ** 2)
    assert np.array_equal(rho == geo["rho_inter"], wedge & ~inclump)
    # clump centres follow Eq. 21 with the r_in offset
    r = np.linalg.norm(geo["centres"], axis=1)
    assert np.all((r >= geo["r_in"]) & (r <= geo["r_out"]))
    lat = np.abs(np.arcsin(geo["centres"][:, 2] / r))
    assert np.all(lat <= math.radians(45.0) + 1e-12)


def test_shell_mass(orc):
    r_in_cells = 3.0
    n = 24
    m = mi.shell(n=n, n_packets=10, ratio=n / 2 / r_in_cells * 0.95)
    geo = m.geometry
    rho = orc.voxelize_shell(n, n, n, m.origin, m.dcell, geo)
    mass = rho.sum() * m.dcell**3
    exact = 4 * math.pi * geo["rho0"] * geo["r_in"] ** 2 * (geo["r_out"] - geo["r_in"])
    assert mass == pytest.approx(exact, rel=0.01)
    c = n // 2
    assert rho[c, c, c] == 0.0  # cavity


def test_constant_shell_mass(orc):
    """power 0: the envelope of the sect. 3.6 run-time comparison holds
    rho0 * 4/3 pi (r_out^3 - r_in^3) (up to the cells its surfaces cut)."""
    m = mi.replica(n=40, n_packets=10, r_out_au=700.0 * 0.95, r_in_au=60.0)
    geo = m.geometry
    assert geo["power"] == 0.0
    rho = orc.voxelize_shell(m.nx, m.ny, m.nz, m.origin, m.dcell, geo)
    mass = rho.sum() * m.dcell**3
    exact = 4 / 3 * math.pi * geo["rho0"] * (geo["r_out"] ** 3 - geo["r_in"] ** 3)
    assert mass == pytest.approx(exact, rel=0.01)
    inside = rho[rho > 0]
    assert np.max(inside) == pytest.approx(geo["rho0"], rel=1e-12)
    c = m.nx // 2
    assert rho[c, c, c] == 0.0


def test_ivezic_dust_law():
    lam = np.array([0.3, 0.55, 1.0, 2.0, 10.0])
    ka, ks, g = mi.ivezic_dust(lam, kext_v=2.0)
    np.testing.assert_allclose(ka[0], [1.0, 1.0, 1.0, 0.5, 0.1], rtol=1e-15)
    np.testing.assert_allclose(ks[0], [1.0, 1.0, 1.0, 0.0625, 1e-4], rtol=1e-15)
    assert np.all(g == 0.0)
