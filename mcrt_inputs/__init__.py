"""Seeded synthetic inputs for the Monte Carlo dust radiative-transfer path.

This module is shared by the CPU oracle (tests) and the HIP library. It only
produces *inputs*: wavelength grids, opacity curves, source spectral shapes,
clump centres and the numbers that name each workload. It contains none of the
transport, temperature or ray-tracing arithmetic; each side computes those on
its own from these inputs.

Workloads (all synthetic, shaped after the paper's models):

* ``cube``   - 32^3 uniform cube, central 5800 K blackbody, one grey-ish
               species (kappa ~ lambda^-1.5, albedo 0.5, g 0.5) on 20 wavelengths
               0.1-1000 um, centre-to-edge V-band tau 1 (sect. 2 method test).
* ``shell``  - 128^3 spherical r^-2 shell between R_in and 1000 R_in around a
               2500 K star of 1 L_sun (the shell of the run-time comparison,
               sect. 3.6, and the 1D benchmark, sect. 5.1), two large-grain
               species with mass fractions 0.68 / 0.32 (sect. 6) on 100 wavelengths.
* ``torus``  - 256^3 clumpy AGN torus (sect. 6): 45 deg half opening,
               r_in 0.4 pc, r_out 6 pc, 2000 clumps of radius 0.02 r_out,
               V-band optical depth 30 through a clump centre, contrast 100,
               broken power-law AGN source (Eq. 20), silicate + carbon + PAH.
* ``batch``  - 64 torus models of uneven size for one batched launch.
* ``images`` - ray-tracer workload on the torus: 512^2 pixels, 16 imaged
               wavelengths, 8 viewing angles 5..85 deg (sect. 6.2).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

AU_CM = 1.495978707e13
PC_CM = 3.0856775814913673e18
LSUN = 3.828e33
MPC_CM = 1e6 * PC_CM

__all__ = [
    "AU_CM", "PC_CM", "LSUN", "MPC_CM", "ModelInputs", "lambda_grid",
    "grey_dust", "silicate_like", "carbon_like", "pah_like", "pah_table",
    "agn_shape", "torus_clumps", "cube", "shell", "torus", "batch_specs",
    "image_views", "workload", "uniform_rho",
]


@dataclasses.dataclass
class ModelInputs:
    """Everything a transport run needs, as plain float64/int arrays.

    Grid: ``nx, ny, nz`` cubic cells of side ``dcell`` [cm] with the low corner
    at ``origin`` [cm]; density ``rho`` [g/cm^3] with shape (nz, ny, nx), x
    fastest, or ``None`` when a voxelizer builds it from ``geometry``.
    Dust: ``lam_um`` increasing; per species mass fraction ``mass_frac`` and
    ``kabs``, ``ksca`` [cm^2 per g of dust], ``g`` with shape (ns, nl).
    Sources: positions [cm], luminosities [erg/s] and either a spectral shape
    proportional to L_nu per wavelength or a blackbody temperature.
    """

    name: str
    nx: int
    ny: int
    nz: int
    origin: np.ndarray
    dcell: float
    rho: Optional[np.ndarray]
    lam_um: np.ndarray
    mass_frac: np.ndarray
    kabs: np.ndarray
    ksca: np.ndarray
    g: np.ndarray
    src_pos: np.ndarray
    src_lum: np.ndarray
    src_shape: Optional[np.ndarray] = None
    src_tbb: Optional[np.ndarray] = None
    pah_species: int = -1
    pah_emis: Optional[np.ndarray] = None
    pah_edges: Optional[np.ndarray] = None
    geometry: Optional[dict] = None
    n_packets: int = 0
    seed: int = 0
    # one level of refinement: ref (nz, ny, nx) uint8, r >= 2 divides a cube
    # into r^3 sub-cubes; rho_sub their densities, cube by cube in linear cube
    # order, x fastest inside a cube
    ref: Optional[np.ndarray] = None
    rho_sub: Optional[np.ndarray] = None

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def nleaf(self) -> int:
        return self.ncells + (0 if self.rho_sub is None else int(self.rho_sub.size))

    @property
    def nl(self) -> int:
        return int(self.lam_um.shape[0])

    @property
    def ns(self) -> int:
        return int(self.mass_frac.shape[0])


# --------------------------------------------------------------------------
# wavelength grids and opacity curves (synthetic recipes; inputs only)
# --------------------------------------------------------------------------

def lambda_grid(n: int, lo_um: float, hi_um: float) -> np.ndarray:
    """n log-spaced wavelengths [um], increasing."""
    return np.geomspace(lo_um, hi_um, n).astype(np.float64)


def _gauss_dex(lam, lc, sig):
    return np.exp(-np.log10(lam / lc) ** 2 / (2.0 * sig * sig))


def grey_dust(lam, kext_v=1.0e4, albedo=0.5, g=0.5, slope=-1.5):
    """One species with kappa_ext = kext_v (lam/0.55)^slope, constant albedo/g."""
    kext = kext_v * (lam / 0.55) ** slope
    ksca = albedo * kext
    kabs = kext - ksca
    return (kabs[None, :].copy(), ksca[None, :].copy(),
            np.full((1, lam.size), g, dtype=np.float64))


def _scaled(kabs_raw, alb, gg, lam_v_raw_ext, kext_v):
    scale = kext_v / lam_v_raw_ext
    kabs = kabs_raw * scale
    ksca = kabs * alb / (1.0 - alb)
    return kabs, ksca, gg


def silicate_like(lam, kext_v=35000.0):
    """Silicate-like curve with 9.7 and 18 um bumps (synthetic)."""
    def raw(l):
        return (l / 0.55) ** -1.5 * (1.0 + 3.0 * _gauss_dex(l, 9.7, 0.06)
                                     + 1.5 * _gauss_dex(l, 18.0, 0.08))
    def alb(l):
        return 0.6 / (1.0 + l * l)
    a_v = alb(np.array([0.55]))[0]
    ext_v = raw(np.array([0.55]))[0] / (1.0 - a_v)
    return _scaled(raw(lam), alb(lam), 0.6 * np.exp(-lam / 2.0), ext_v, kext_v)


def carbon_like(lam, kext_v=35000.0):
    """Carbon-like curve with a 2175 A bump (synthetic)."""
    def raw(l):
        return (l / 0.55) ** -1.0 * (1.0 + 0.5 * _gauss_dex(l, 0.2175, 0.05))
    def alb(l):
        return 0.35 / (1.0 + l * l)
    a_v = alb(np.array([0.55]))[0]
    ext_v = raw(np.array([0.55]))[0] / (1.0 - a_v)
    return _scaled(raw(lam), alb(lam), 0.5 * np.exp(-lam / 2.0), ext_v, kext_v)


def pah_like(lam, kabs_v=35000.0):
    """Pure absorber with a UV-rising cross section (synthetic PAH)."""
    kabs = kabs_v * np.exp(-(lam - 0.55) / 0.5)
    return kabs, np.zeros_like(lam), np.zeros_like(lam)


def pah_table(lam, rows: int = 8):
    """PAH emissivity rows eps_n(nu) on the grid plus the row edges.

    Rows are selected by the absorbed PAH power per unit PAH mass and steradian
    [erg/s/g/sr]; ``edges`` has rows-1 increasing entries.
    """
    bands = [(3.3, 1.0), (6.2, 3.0), (7.7, 6.0), (8.6, 2.0), (11.3, 4.0), (12.7, 2.0)]
    emis = np.zeros((rows, lam.size))
    for r in range(rows):
        e = np.zeros_like(lam)
        for lc, wt in bands:
            e += wt * _gauss_dex(lam, lc, 0.02)
        e += 0.1 * (r + 1) * _gauss_dex(lam, 15.0, 0.3)
        emis[r] = e
    edges = np.geomspace(1e4, 1e10, rows - 1)
    return emis, edges


def agn_shape(lam):
    """L_nu shape of the broken power law of Eq. 20 (lambda F_lambda given).

    lambda F_lambda ~ lambda^1.2 (<0.01 um), const (0.01-0.1), lambda^-0.5
    (0.1-1), lambda^-3 (>1), continuous at the breaks; L_nu ~ lambda (lambda F_lambda).
    """
    lf = np.where(lam < 0.01, (lam / 0.01) ** 1.2,
         np.where(lam < 0.1, 1.0,
         np.where(lam < 1.0, (lam / 0.1) ** -0.5, 10.0 ** -0.5 * lam ** -3.0)))
    return lf * lam


def uniform_rho(n: int, value: float) -> np.ndarray:
    return np.full((n, n, n), value, dtype=np.float64)


# --------------------------------------------------------------------------
# geometry draws
# --------------------------------------------------------------------------

def torus_clumps(n_clumps: int, seed: int, r_in: float, r_out: float,
                 theta1_deg: float) -> np.ndarray:
    """Clump centres (n, 3) [cm] following Eq. 21 with the r_in offset.

    r = r_in + z1 (r_out - r_in), phi = 2 pi z2, theta = pi/2 + (2 z3 - 1) theta1.
    """
    rng = np.random.Generator(np.random.Philox(key=seed))
    z = rng.random((n_clumps, 3))
    th1 = math.radians(theta1_deg)
    r = r_in + z[:, 0] * (r_out - r_in)
    phi = 2.0 * math.pi * z[:, 1]
    th = 0.5 * math.pi + (2.0 * z[:, 2] - 1.0) * th1
    return np.stack([r * np.sin(th) * np.cos(phi), r * np.sin(th) * np.sin(phi),
                     r * np.cos(th)], axis=1)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def cube(n: int = 32, n_packets: int = 100_000, seed: int = 0, tau_v: float = 1.0,
         half_au: float = 10.0, nl: int = 20, albedo: float = 0.5, g: float = 0.5,
         kext_v: float = 1.0e4, t_star: float = 5800.0) -> ModelInputs:
    """Uniform cube with a blackbody point source on the central vertex."""
    lam = lambda_grid(nl, 0.1, 1000.0)
    kabs, ksca, gg = grey_dust(lam, kext_v=kext_v, albedo=albedo, g=g)
    half = half_au * AU_CM
    rho0 = tau_v / (kext_v * half)
    return ModelInputs(
        name=f"cube{n}", nx=n, ny=n, nz=n, origin=np.array([-half] * 3),
        dcell=2.0 * half / n, rho=uniform_rho(n, rho0), lam_um=lam,
        mass_frac=np.array([1.0]), kabs=kabs, ksca=ksca, g=gg,
        src_pos=np.zeros((1, 3)), src_lum=np.array([LSUN]), src_shape=None,
        src_tbb=np.array([t_star]), n_packets=n_packets, seed=seed,
        geometry={"kind": "cube", "rho": rho0})


def shell(n: int = 128, tau_v: float = 10.0, n_packets: int = 10_000_000,
          seed: int = 0, nl: int = 100, r_in_au: float = 1.0,
          ratio: float = 1000.0, t_star: float = 2500.0) -> ModelInputs:
    """r^-2 shell R_in..ratio*R_in in a box of half-size ratio*R_in."""
    lam = lambda_grid(nl, 0.1, 1000.0)
    s = silicate_like(lam)
    c = carbon_like(lam)
    r_in = r_in_au * AU_CM
    r_out = ratio * r_in
    kext_v = 35000.0
    rho0 = tau_v / (kext_v * r_in * (1.0 - r_in / r_out))
    half = r_out
    return ModelInputs(
        name=f"shell{n}_tau{tau_v:g}", nx=n, ny=n, nz=n, origin=np.array([-half] * 3),
        dcell=2.0 * half / n, rho=None, lam_um=lam, mass_frac=np.array([0.68, 0.32]),
        kabs=np.stack([s[0], c[0]]), ksca=np.stack([s[1], c[1]]), g=np.stack([s[2], c[2]]),
        src_pos=np.zeros((1, 3)), src_lum=np.array([LSUN]), src_tbb=np.array([t_star]),
        n_packets=n_packets, seed=seed,
        geometry={"kind": "shell", "rho0": rho0, "r_in": r_in, "r_out": r_out})


def ivezic_dust(lam, kext_v=1.0e4, lam0=1.0):
    """Grey-to-power-law grains of the 1D benchmark (sect. 5.1): q_abs = q_sca =
    1 below lam0, q_abs = lam0/lam and q_sca = (lam0/lam)^4 above; isotropic
    scattering. Scaled so that kappa_ext at 0.55 um is kext_v."""
    x = np.minimum(1.0, lam0 / np.asarray(lam, dtype=np.float64))
    qa, qs = x, x**4
    scale = kext_v / 2.0  # both efficiencies are 1 at 0.55 um
    return (scale * qa)[None, :], (scale * qs)[None, :], np.zeros((1, len(lam)))


def replica(n: int = 100, tau_v: float = 10.0, n_packets: int = 10_000_000, seed: int = 0,
            nl: int = 100, r_in_au: float = 0.7, r_out_au: float = 700.0,
            t_star: float = 2500.0) -> ModelInputs:
    """Run-time comparison model of sect. 3.6 (Table 1): a 2500 K, 1 L_sun star
    in a constant-density envelope 0.7-700 AU with tau_V = 10 from the star to
    the outer edge, 10^6 cells (box of half-size r_out), 10^7 packets."""
    lam = lambda_grid(nl, 0.1, 1000.0)
    kext_v = 1.0e4
    kabs, ksca, gg = ivezic_dust(lam, kext_v=kext_v)
    r_in, r_out = r_in_au * AU_CM, r_out_au * AU_CM
    rho0 = tau_v / (kext_v * (r_out - r_in))
    return ModelInputs(
        name=f"replica{n}", nx=n, ny=n, nz=n, origin=np.array([-r_out] * 3),
        dcell=2.0 * r_out / n, rho=None, lam_um=lam, mass_frac=np.array([1.0]),
        kabs=kabs, ksca=ksca, g=gg, src_pos=np.zeros((1, 3)), src_lum=np.array([LSUN]),
        src_tbb=np.array([t_star]), n_packets=n_packets, seed=seed,
        geometry={"kind": "shell", "rho0": rho0, "r_in": r_in, "r_out": r_out, "power": 0.0})


def torus(n: int = 256, n_clumps: int = 2000, n_packets: int = 100_000_000,
          seed: int = 0, geo_seed: int = 2, nl: int = 100, lum: float = 1e45,
          r_in_pc: float = 0.4, r_out_pc: float = 6.0, theta1_deg: float = 45.0,
          clump_frac: float = 0.02, tau_clump: float = 30.0, contrast: float = 100.0,
          pah: bool = True, pah_frac: float = 0.05) -> ModelInputs:
    """Clumpy AGN torus of sect. 6 on an n^3 grid spanning +-r_out."""
    lam = lambda_grid(nl, 0.01, 1000.0)
    s = silicate_like(lam)
    c = carbon_like(lam)
    r_in = r_in_pc * PC_CM
    r_out = r_out_pc * PC_CM
    r_cl = clump_frac * r_out
    kext_v = 35000.0
    rho_cl = tau_clump / (kext_v * 2.0 * r_cl)
    centres = torus_clumps(n_clumps, geo_seed, r_in, r_out, theta1_deg)
    kabs = [s[0], c[0]]
    ksca = [s[1], c[1]]
    gg = [s[2], c[2]]
    frac = [0.68, 0.32]
    pah_species = -1
    emis = edges = None
    if pah:
        p = pah_like(lam)
        kabs.append(p[0]); ksca.append(p[1]); gg.append(p[2])
        frac = [0.68 * (1 - pah_frac), 0.32 * (1 - pah_frac), pah_frac]
        pah_species = 2
        emis, edges = pah_table(lam)
    th1 = math.radians(theta1_deg)
    return ModelInputs(
        name=f"torus{n}", nx=n, ny=n, nz=n, origin=np.array([-r_out] * 3),
        dcell=2.0 * r_out / n, rho=None, lam_um=lam, mass_frac=np.array(frac),
        kabs=np.stack(kabs), ksca=np.stack(ksca), g=np.stack(gg),
        src_pos=np.zeros((1, 3)), src_lum=np.array([lum]), src_shape=agn_shape(lam)[None, :],
        pah_species=pah_species, pah_emis=emis, pah_edges=edges,
        n_packets=n_packets, seed=seed,
        geometry={"kind": "torus", "centres": centres, "r_clump": r_cl,
                  "rho_clump": rho_cl, "rho_inter": rho_cl / contrast,
                  "r_in": r_in, "r_out": r_out, "sin_theta1": math.sin(th1)})


def batch_specs(n_models: int = 64, seed: int = 4) -> List[dict]:
    """Uneven torus models: grid 64..192 step 8, 200..1e4 clumps (log-uniform),
    40..100 wavelengths, 1e6..1e7 packets (log-uniform, rounded to 1e4)."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    out = []
    for m in range(n_models):
        n = int(rng.integers(0, 17)) * 8 + 64
        ncl = int(round(10 ** rng.uniform(math.log10(200), 4.0)))
        nl = int(rng.integers(40, 101))
        npk = int(round(10 ** rng.uniform(6.0, 7.0) / 1e4)) * 10_000
        out.append({"n": n, "n_clumps": ncl, "nl": nl, "n_packets": npk,
                    "seed": m, "geo_seed": 1000 + m})
    return out


def sub_offsets(ref: np.ndarray) -> np.ndarray:
    """First sub-cube of each cube: exclusive prefix sum of r^3 over the
    divided cubes (r >= 2), in linear cube order (the layout of rho_sub)."""
    r = np.asarray(ref, dtype=np.int64).ravel()
    n = np.where(r >= 2, r**3, 0)
    return np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)


def refine_random(m: ModelInputs, frac: float = 0.3, rmax: int = 3, seed: int = 0,
                  spread: float = 1.0) -> ModelInputs:
    """Divide a random share of the cubes of a model with explicit densities
    into r^3 sub-cubes (r uniform in 2..rmax) whose densities scatter
    log-normally (sigma `spread`) about the cube's (seeded; inputs only)."""
    rng = np.random.Generator(np.random.Philox(key=1000 + seed))
    nc = m.ncells
    ref = np.where(rng.random(nc) < frac, rng.integers(2, rmax + 1, nc), 0).astype(np.uint8)
    rho = np.asarray(m.rho, dtype=np.float64).ravel()
    subs = []
    for c in np.flatnonzero(ref):
        r = int(ref[c])
        subs.append(rho[c] * np.exp(spread * rng.normal(size=r**3)))
    rho_sub = np.concatenate(subs) if subs else np.zeros(0)
    return dataclasses.replace(m, ref=ref.reshape(m.nz, m.ny, m.nx), rho_sub=rho_sub,
                               name=m.name + "_refined")


def image_views(n_views: int = 8, n_img: int = 16, nl: int = 100):
    """Viewing angles (theta 5..85 deg, phi 0) and imaged wavelength indices."""
    th = [5.0 + k * 80.0 / (n_views - 1) for k in range(n_views)] if n_views > 1 else [45.0]
    views = np.array([[t, 0.0] for t in th])
    idx = np.array([int(round(k * (nl - 1) / (n_img - 1))) for k in range(n_img)],
                   dtype=np.int32)
    return views, idx


def workload(name: str, **kw) -> ModelInputs:
    return {"cube": cube, "shell": shell, "torus": torus, "replica": replica}[name](**kw)
