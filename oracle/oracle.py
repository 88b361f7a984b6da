"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use this module. It never touches the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "mcrt_oracle.c")

FROZEN, BW_EPOCH = 0, 1
SCAT_HG, SCAT_GFACTOR = 0, 1
TAU_FLIGHT, TAU_PER_CELL = 0, 1
RT_EXT, RT_ABS_LITERAL = 0, 1
ESCAPED, KILLED, PAH_STOP = 1, 2, 3

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


def build(force: bool = True, out: str = None, native: bool = False,
          sanitize: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no contraction, no value-changing
    optimisation). native=True adds -O3 -march=native for timing on the
    machine that runs it (same IEEE arithmetic, written to `out`).
    sanitize=True builds with AddressSanitizer and UndefinedBehaviorSanitizer
    (every report fatal); the process that loads it must preload libasan."""
    path = out or LIB_PATH
    if force or not os.path.exists(path):
        opt = ["-O3", "-march=native"] if native else ["-O2"]
        if sanitize:
            opt = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                   "-fno-sanitize-recover=all"]
        cmd = ["gcc", *opt, "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-o", path, SRC, "-lm"]
        subprocess.check_call(cmd, cwd=HERE)
    return path


def use_library(path: str) -> None:
    """Load the oracle from another build of the same source (see build)."""
    global LIB_PATH, _lib
    LIB_PATH = path
    _lib = None


class Model(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("pad0", C.c_int32),
        ("origin", C.c_double * 3), ("dcell", C.c_double), ("rho", _dp),
        ("nl", C.c_int32), ("ns", C.c_int32), ("lam_um", _dp), ("mass_frac", _dp),
        ("kabs", _dp), ("ksca", _dp), ("g", _dp),
        ("pah_species", C.c_int32), ("n_pah_rows", C.c_int32), ("pah_emis", _dp),
        ("pah_edges", _dp), ("nsrc", C.c_int32), ("scat_law", C.c_int32), ("src_pos", _dp),
        ("src_lum", _dp), ("src_shape", _dp), ("src_tbb", _dp),
        ("nview", C.c_int32), ("nimg", C.c_int32), ("view_deg", _dp), ("img_idx", _ip),
        ("distance", C.c_double), ("ref", C.POINTER(C.c_uint8)),
        ("sub_off", C.POINTER(C.c_int64)), ("rho_sub", _dp), ("nsub", C.c_int64),
    ]


class Opts(C.Structure):
    _fields_ = [
        ("mode", C.c_int32), ("n_iter", C.c_int32), ("epoch", C.c_uint64),
        ("n_total", C.c_uint64), ("lucy_tau", C.c_double), ("mrw_tau", C.c_double),
        ("mrw_gamma", C.c_double), ("max_int", C.c_uint64), ("ntheta", C.c_int32),
        ("model_id", C.c_int32), ("record", C.c_int32), ("tau_mode", C.c_int32),
        ("src_strata", C.c_uint64), ("pah_nc", C.c_double), ("pah_tcool", C.c_double),
        ("sh_order", C.c_int32), ("pad2", C.c_int32),
    ]


class Record(C.Structure):
    _fields_ = [
        ("pid", C.c_uint64), ("pos", C.c_double * 3), ("dir", C.c_double * 3),
        ("j", C.c_int32), ("status", C.c_int32), ("weight", C.c_double),
        ("n_cross", C.c_uint64), ("n_scat", C.c_uint64), ("n_abs", C.c_uint64),
        ("n_mrw", C.c_uint64), ("n_lucy", C.c_uint64), ("min_margin", C.c_double),
    ]


RECORD_DTYPE = np.dtype([
    ("pid", "<u8"), ("pos", "<f8", (3,)), ("dir", "<f8", (3,)), ("j", "<i4"),
    ("status", "<i4"), ("weight", "<f8"), ("n_cross", "<u8"), ("n_scat", "<u8"),
    ("n_abs", "<u8"), ("n_mrw", "<u8"), ("n_lucy", "<u8"), ("min_margin", "<f8"),
])
assert RECORD_DTYPE.itemsize == C.sizeof(Record)

STAT_NAMES = ["packets", "escaped", "killed", "pah_stopped", "crossings", "scatters",
              "absorptions", "mrw_steps", "lucy_deposits", "clamped_T"]


class Stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in STAT_NAMES]


class State(C.Structure):
    _fields_ = [
        ("k", C.POINTER(C.c_uint64)), ("epath", _dp), ("T", _dp), ("esnap", _dp),
        ("tt", _dp), ("tvalid", C.POINTER(C.c_uint8)), ("kpah", C.POINTER(C.c_uint32)),
        ("sed", C.POINTER(C.c_uint64)), ("ssca", _dp), ("sh", _dp), ("rec", C.POINTER(Record)),
        ("st", Stats),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        u32p = C.POINTER(C.c_uint32)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_u24.argtypes = [C.c_uint32]; L.orc_u24.restype = C.c_double
        L.orc_draw.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64]
        L.orc_draw.restype = C.c_double
        L.orc_freq_grid.argtypes = [C.c_int, _dp, _dp, _dp]
        for f in ("orc_planck", "orc_dplanck_dT", "orc_hg_mu", "orc_hg_phase"):
            getattr(L, f).argtypes = [C.c_double, C.c_double]
            getattr(L, f).restype = C.c_double
        for f in ("orc_mrw_survival", "orc_mrw_solve"):
            getattr(L, f).argtypes = [C.c_double]
            getattr(L, f).restype = C.c_double
        L.orc_phi.argtypes = [C.POINTER(Model), C.c_int, C.c_double]; L.orc_phi.restype = C.c_double
        L.orc_invert_T.argtypes = [C.POINTER(Model), C.c_int, C.c_double]
        L.orc_invert_T.restype = C.c_double
        L.orc_rosseland.argtypes = [C.POINTER(Model), C.c_double]
        L.orc_rosseland.restype = C.c_double
        L.orc_planck_mean.argtypes = [C.POINTER(Model), C.c_int, C.c_double]
        L.orc_planck_mean.restype = C.c_double
        L.orc_dda.argtypes = [C.POINTER(Model), _dp, _dp, C.c_int, C.POINTER(C.c_int64), _dp]
        L.orc_init_T.argtypes = [C.POINTER(Model), _dp]
        L.orc_nleaf.argtypes = [C.POINTER(Model)]
        L.orc_nleaf.restype = C.c_int64
        L.orc_leaf_box.argtypes = [C.POINTER(Model), C.c_int64, _dp, _dp, _dp]
        L.orc_ylm.argtypes = [C.c_int, _dp, _dp]
        L.orc_sh_view_sums.argtypes = [C.POINTER(Model), C.c_int, _dp, _dp, _dp]
        L.orc_pah_dissociates.argtypes = [C.POINTER(Model), C.POINTER(Opts), C.c_uint32,
                                          C.c_int64]
        L.orc_run.argtypes = [C.POINTER(Model), C.POINTER(Opts), C.c_uint64, C.c_uint64,
                              C.c_uint64, C.POINTER(State)]
        L.orc_pah_pass.argtypes = [C.POINTER(Model), C.POINTER(Opts), C.c_uint64, C.POINTER(State)]
        L.orc_finalize_T.argtypes = [C.POINTER(Model), C.POINTER(Opts), C.POINTER(State)]
        L.orc_raytrace.argtypes = [C.POINTER(Model), C.c_int, _dp, _dp, _dp, C.c_int, C.c_int,
                                   _dp, _dp]
        L.orc_raytrace_adjoint.argtypes = [C.POINTER(Model), C.c_int, _dp, _dp, _dp, C.c_int,
                                           C.c_int, _dp, _dp, _dp]
        L.orc_voxelize_torus.argtypes = [C.c_int, C.c_int, C.c_int, _dp, C.c_double, C.c_int,
                                         _dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                         C.c_double, C.c_double, _dp]
        L.orc_voxelize_shell.argtypes = [C.c_int, C.c_int, C.c_int, _dp, C.c_double, C.c_double,
                                         C.c_double, C.c_double, C.c_double, _dp]
        _lib = L
    return _lib


def _p(a, t=C.c_double):
    if a is None:
        return C.cast(None, C.POINTER(t))
    return a.ctypes.data_as(C.POINTER(t))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- scalars

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def u24(x):
    return lib().orc_u24(x)


def draw(seed, pid, it, model, tag, d):
    return lib().orc_draw(seed, pid, it, model, tag, d)


def freq_grid(lam):
    lam = _f64(lam)
    nu = np.empty_like(lam)
    w = np.empty_like(lam)
    lib().orc_freq_grid(lam.size, _p(lam), _p(nu), _p(w))
    return nu, w


def planck(nu, T):
    return lib().orc_planck(nu, T)


def dplanck_dT(nu, T):
    return lib().orc_dplanck_dT(nu, T)


def hg_mu(g, u):
    return lib().orc_hg_mu(g, u)


def hg_phase(g, mu):
    return lib().orc_hg_phase(g, mu)


def mrw_survival(y):
    return lib().orc_mrw_survival(y)


def mrw_solve(u):
    return lib().orc_mrw_solve(u)


def ylm(lmax, d):
    """Real orthonormal spherical harmonics at unit vector d, index l^2 + l + m."""
    y = np.zeros((lmax + 1) ** 2)
    lib().orc_ylm(lmax, _p(_f64(d)), _p(y))
    return y


def voxelize_torus(nx, ny, nz, origin, dcell, geo):
    rho = np.zeros((nz, ny, nx))
    cen = _f64(geo["centres"])
    o = _f64(origin)
    lib().orc_voxelize_torus(nx, ny, nz, _p(o), dcell, cen.shape[0], _p(cen), geo["r_clump"],
                             geo["rho_clump"], geo["rho_inter"], geo["r_in"], geo["r_out"],
                             geo["sin_theta1"], _p(rho))
    return rho


def voxelize_shell(nx, ny, nz, origin, dcell, geo):
    rho = np.zeros((nz, ny, nx))
    o = _f64(origin)
    lib().orc_voxelize_shell(nx, ny, nz, _p(o), dcell, geo["rho0"], geo["r_in"], geo["r_out"],
                             geo.get("power", 2.0), _p(rho))
    return rho


def density(mi):
    """Density of a workload: given, or voxelized by the oracle."""
    if mi.rho is not None:
        return _f64(mi.rho)
    kind = mi.geometry["kind"]
    if kind == "torus":
        return voxelize_torus(mi.nx, mi.ny, mi.nz, mi.origin, mi.dcell, mi.geometry)
    if kind == "shell":
        return voxelize_shell(mi.nx, mi.ny, mi.nz, mi.origin, mi.dcell, mi.geometry)
    raise ValueError(kind)


# ------------------------------------------------------------------ model

class Oracle:
    """One model held as C structs plus the numpy arrays they point into."""

    def __init__(self, mi, rho=None, views=None, img_idx=None, distance=1.0, ntheta=10,
                 scat_law=0):
        self.mi = mi
        self.rho = _f64(rho) if rho is not None else density(mi)
        self.lam = _f64(mi.lam_um)
        self.frac = _f64(mi.mass_frac)
        self.kabs = _f64(mi.kabs)
        self.ksca = _f64(mi.ksca)
        self.g = _f64(mi.g)
        self.src_pos = _f64(mi.src_pos)
        self.src_lum = _f64(mi.src_lum)
        self.src_shape = _f64(mi.src_shape)
        self.src_tbb = _f64(mi.src_tbb)
        self.pah_emis = _f64(mi.pah_emis)
        self.pah_edges = _f64(mi.pah_edges)
        self.views = _f64(views) if views is not None else np.zeros((0, 2))
        self.img_idx = (np.ascontiguousarray(img_idx, dtype=np.int32)
                        if img_idx is not None else np.zeros(0, dtype=np.int32))
        self.ntheta = ntheta
        m = Model()
        m.nx, m.ny, m.nz = mi.nx, mi.ny, mi.nz
        for k in range(3):
            m.origin[k] = float(mi.origin[k])
        m.dcell = float(mi.dcell)
        m.rho = _p(self.rho)
        m.nl, m.ns = self.lam.size, self.frac.size
        m.lam_um, m.mass_frac = _p(self.lam), _p(self.frac)
        m.kabs, m.ksca, m.g = _p(self.kabs), _p(self.ksca), _p(self.g)
        m.pah_species = mi.pah_species
        m.n_pah_rows = 0 if self.pah_emis is None else self.pah_emis.shape[0]
        m.pah_emis, m.pah_edges = _p(self.pah_emis), _p(self.pah_edges)
        m.nsrc = self.src_lum.size
        m.src_pos, m.src_lum = _p(self.src_pos), _p(self.src_lum)
        m.src_shape, m.src_tbb = _p(self.src_shape), _p(self.src_tbb)
        m.nview, m.nimg = self.views.shape[0], self.img_idx.size
        m.view_deg = _p(self.views)
        m.img_idx = _p(self.img_idx, C.c_int32)
        m.distance = float(distance)
        m.scat_law = scat_law
        self.ref = self.sub_off = self.rho_sub = None
        if getattr(mi, "ref", None) is not None:
            self.ref = np.ascontiguousarray(mi.ref, dtype=np.uint8).ravel()
            r = self.ref.astype(np.int64)
            n = np.where(r >= 2, r**3, 0)
            self.sub_off = np.ascontiguousarray(np.concatenate([[0], np.cumsum(n)[:-1]]),
                                                dtype=np.int64)
            self.rho_sub = _f64(mi.rho_sub)
            assert self.rho_sub.size == int(n.sum())
            m.ref = _p(self.ref, C.c_uint8)
            m.sub_off = _p(self.sub_off, C.c_int64)
            m.rho_sub = _p(self.rho_sub)
            m.nsub = self.rho_sub.size
        self.m = m
        self.reset()

    @property
    def ncells(self):
        """Leaf cells: cubes plus sub-cubes."""
        return self.mi.nx * self.mi.ny * self.mi.nz + (0 if self.rho_sub is None
                                                        else self.rho_sub.size)

    def reset(self):
        nc, ns, nl = self.ncells, self.frac.size, self.lam.size
        self.k = np.zeros((ns, nc), dtype=np.uint64)
        self.epath = np.zeros((ns, nc))
        self.T = np.zeros((ns, nc))
        self.esnap = np.zeros((ns, nc))
        self.tt = np.zeros((ns, nc))
        self.tvalid = np.zeros((ns, nc), dtype=np.uint8)
        self.kpah = np.zeros(nc, dtype=np.uint32)
        self.sed = np.zeros((self.ntheta, nl), dtype=np.uint64)
        nv, ni = self.views.shape[0], self.img_idx.size
        self.ssca = np.zeros((nv, ni, nc)) if nv * ni > 0 else np.zeros(1)
        self.records = None
        self.sh = None
        self.stats = {n: 0 for n in STAT_NAMES}

    def _state(self, nrec):
        s = State()
        s.k = _p(self.k, C.c_uint64)
        s.epath = _p(self.epath)
        s.T = _p(self.T)
        s.esnap = _p(self.esnap)
        s.tt = _p(self.tt)
        s.tvalid = _p(self.tvalid, C.c_uint8)
        s.kpah = _p(self.kpah, C.c_uint32)
        s.sed = _p(self.sed, C.c_uint64)
        s.ssca = _p(self.ssca)
        s.sh = _p(self.sh)
        if nrec:
            self.records = np.zeros(nrec, dtype=RECORD_DTYPE)
            s.rec = C.cast(self.records.ctypes.data, C.POINTER(Record))
        else:
            s.rec = C.cast(None, C.POINTER(Record))
        return s

    def opts(self, mode=BW_EPOCH, n_iter=3, epoch=4096, n_total=None, lucy_tau=1e-2,
             mrw_tau=0.0, mrw_gamma=2.0, max_int=10_000_000, model_id=0, record=False,
             tau_mode=TAU_FLIGHT, src_strata=0, pah_nc=0.0, pah_tcool=0.0, sh_order=0):
        o = Opts()
        o.tau_mode, o.src_strata = tau_mode, src_strata
        o.pah_nc, o.pah_tcool = pah_nc, pah_tcool
        if not 0 <= sh_order <= 16:
            raise ValueError("sh_order must be 0..16")
        o.sh_order = sh_order
        ni = self.img_idx.size
        if sh_order > 0 and (self.sh is None or self.sh.shape[1] != sh_order**2):
            self.sh = np.zeros((ni, sh_order**2, self.ncells))
        o.mode, o.n_iter, o.epoch = mode, n_iter, epoch
        o.n_total = n_total if n_total is not None else self.mi.n_packets
        o.lucy_tau, o.mrw_tau, o.mrw_gamma = lucy_tau, mrw_tau, mrw_gamma
        o.max_int, o.ntheta, o.model_id, o.record = max_int, self.ntheta, model_id, int(record)
        return o

    def _collect(self, st):
        for n in STAT_NAMES:
            self.stats[n] += getattr(st.st, n)

    def init_T(self):
        lib().orc_init_T(C.byref(self.m), _p(self.T))

    def run(self, first=0, n=None, seed=None, **kw):
        n = self.mi.n_packets if n is None else n
        seed = self.mi.seed if seed is None else seed
        o = self.opts(**kw)
        st = self._state(n if o.record else 0)
        lib().orc_run(C.byref(self.m), C.byref(o), first, n, seed, C.byref(st))
        self._collect(st)
        return self

    def pah_pass(self, seed=None, **kw):
        seed = self.mi.seed if seed is None else seed
        o = self.opts(**kw)
        npk = int(self.kpah.sum())
        st = self._state(npk if o.record else 0)
        lib().orc_pah_pass(C.byref(self.m), C.byref(o), seed, C.byref(st))
        self._collect(st)
        return self

    def finalize(self, **kw):
        o = self.opts(**kw)
        st = self._state(0)
        lib().orc_finalize_T(C.byref(self.m), C.byref(o), C.byref(st))
        self._collect(st)
        return self.T

    def energy(self, n_total=None):
        xi = self.xi(n_total)
        return self.k.astype(np.float64) * xi + self.epath

    def xi(self, n_total=None):
        n_total = self.mi.n_packets if n_total is None else n_total
        return float(np.sum(self.src_lum)) / n_total

    def sh_view_sums(self, k, sh=None):
        """Scattered-light sums [img][cells] toward unit vector k from the
        moments of the last run with sh_order > 0."""
        sh = self.sh if sh is None else _f64(sh)
        out = np.zeros((self.img_idx.size, self.ncells))
        lib().orc_sh_view_sums(C.byref(self.m), int(round(np.sqrt(sh.shape[1]))), _p(sh),
                               _p(_f64(k)), _p(out))
        return out

    def leaf_box(self, leaf):
        """(lower corner, edge, density) of a leaf cell."""
        lo = np.zeros(3)
        h, r = np.zeros(1), np.zeros(1)
        lib().orc_leaf_box(C.byref(self.m), int(leaf), _p(lo), _p(h), _p(r))
        return lo, float(h[0]), float(r[0])

    def pah_dissociates(self, kpah=None, **kw):
        """Eq. 8 decision per cell for the given pass-1 PAH counts."""
        kp = self.kpah if kpah is None else kpah
        o = self.opts(**kw)
        return np.array([lib().orc_pah_dissociates(C.byref(self.m), C.byref(o), int(kp[c]), c)
                         for c in range(self.ncells)], dtype=bool)

    def phi(self, s, T):
        return lib().orc_phi(C.byref(self.m), s, T)

    def invert_T(self, s, rhs):
        return lib().orc_invert_T(C.byref(self.m), s, rhs)

    def rosseland(self, T):
        """Rosseland mean of the mixture extinction at T [cm^2/g]."""
        return lib().orc_rosseland(C.byref(self.m), T)

    def planck_mean(self, s, T):
        """Planck mean of species s absorption at T [cm^2/g]."""
        return lib().orc_planck_mean(C.byref(self.m), s, T)

    def dda(self, p0, d, maxseg=10000):
        p0 = _f64(p0)
        d = _f64(d)
        cells = np.zeros(maxseg, dtype=np.int64)
        lens = np.zeros(maxseg)
        n = lib().orc_dda(C.byref(self.m), _p(p0), _p(d), maxseg, _p(cells, C.c_int64), _p(lens))
        if n < 0:
            raise RuntimeError("maxseg too small")
        return cells[:n], lens[:n]

    def raytrace(self, npx, npy, T=None, ssca=None, rho_rt=None, rt_mode=RT_EXT):
        """Images [view][img][npy][npx] and SED [view][img]; rho_rt replaces the
        density in the optical depths only (source functions keep the model's)."""
        T = _f64(self.T if T is None else T)
        nv, ni = self.views.shape[0], self.img_idx.size
        img = np.zeros((nv, ni, npy, npx))
        sed = np.zeros((nv, ni))
        ss = None if ssca is None else _f64(ssca)
        rr = None if rho_rt is None else _f64(rho_rt)
        lib().orc_raytrace(C.byref(self.m), rt_mode, _p(T), _p(ss), _p(rr), npx, npy, _p(img),
                           _p(sed))
        return img, sed

    def raytrace_adjoint(self, npx, npy, w_img=None, w_sed=None, T=None, ssca=None, rho_rt=None,
                         rt_mode=RT_EXT):
        T = _f64(self.T if T is None else T)
        ss = None if ssca is None else _f64(ssca)
        rr = None if rho_rt is None else _f64(rho_rt)
        drho = np.zeros(self.ncells)
        lib().orc_raytrace_adjoint(C.byref(self.m), rt_mode, _p(T), _p(ss), _p(rr), npx, npy,
                                   _p(_f64(w_img)), _p(_f64(w_sed)), _p(drho))
        return drho
