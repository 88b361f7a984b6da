"""The library's scattering rotation (Eq. 15 angle about the incoming
direction), built for the host from the same header the kernels use.

In FP32, directions within ~2e-4 rad of the z axis have d_z == 1.0f exactly;
the rotation must still return a finite unit vector at angle acos(mu) from d
with a uniform azimuth, in both precisions."""
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def probe():
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "scatter_probe")
    subprocess.check_call(["hipcc", "-O2", "--offload-arch=gfx950", "-ffp-contract=off", "-o", exe,
                           os.path.join(HERE, "scatter_probe.cpp")])
    return exe


def rotate(probe, prec, d, mu, phi):
    lines = "".join(f"{prec} {float(x[0]).hex()} {float(x[1]).hex()} {float(x[2]).hex()} "
                    f"{float(m).hex()} {float(p).hex()}\n"
                    for x, m, p in zip(d, mu, phi))
    out = subprocess.run([probe], input=lines, capture_output=True, text=True, check=True).stdout
    return np.array([[float.fromhex(v) for v in ln.split()] for ln in out.strip().splitlines()])


def unit(v, prec):
    """v normalised in the given precision (4 or 8 bytes), as float64."""
    if prec == 8:
        v = np.asarray(v, dtype=np.float64)
        return v / np.linalg.norm(v)
    v = np.asarray(v, dtype=np.float32)
    return (v / np.float32(np.sqrt(np.sum(v.astype(np.float64) ** 2)))).astype(np.float64)


@pytest.mark.parametrize("prec", [4, 8])
def test_rotation_near_and_at_the_poles(probe, prec):
    dirs = [np.array([0.0, 0.0, 1.0]), np.array([0.0, 0.0, -1.0]),
            unit([1e-4, 5e-5, 1.0], prec), unit([-3e-5, 2e-4, -1.0], prec),
            unit([1e-3, -2e-3, 1.0], prec), unit([0.6, -0.48, 0.64], prec)]
    if prec == 4:
        assert np.float32(dirs[2][2]) == 1.0  # rounds onto the pole in FP32
    rng = np.random.default_rng(1)
    n = 400
    for d in dirs:
        mu = rng.uniform(-1, 1, n)
        phi = rng.uniform(0, 2 * math.pi, n)
        out = rotate(probe, prec, [d] * n, mu, phi)
        assert np.all(np.isfinite(out)), d
        tol = 2e-6 if prec == 4 else 1e-13
        np.testing.assert_allclose(np.linalg.norm(out, axis=1), 1.0, atol=tol)
        # the polar angle from d is acos(mu)
        tol = 5e-4 if prec == 4 else 1e-9
        np.testing.assert_allclose(out @ d, mu, atol=tol)


@pytest.mark.parametrize("prec", [4, 8])
def test_rotation_azimuth_is_uniform(probe, prec):
    """For fixed mu and phi on a uniform grid the new directions average to
    mu d (the perpendicular parts cancel only if the azimuthal frame is
    orthonormal), also for a direction that is the pole in FP32."""
    d = unit([1e-4, 5e-5, 1.0], prec)
    mu = 0.3
    phi = (np.arange(720) + 0.5) * (2 * math.pi / 720)
    out = rotate(probe, prec, [d] * phi.size, [mu] * phi.size, phi)
    np.testing.assert_allclose(out.mean(axis=0), mu * d, atol=3e-6)
    # second moments: the perpendicular part has variance (1 - mu^2)/2 per axis
    perp = out - (out @ d)[:, None] * d
    cov = perp.T @ perp / phi.size
    assert np.trace(cov) == pytest.approx(1 - mu * mu, rel=1e-4)
