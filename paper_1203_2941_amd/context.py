"""Python front end of one libmcrt context (argument marshalling only).

Host arrays are numpy; device buffers are torch tensors on the context's GPU
(PyTorch provides device memory and streams; every step of the method runs
in the library's kernels).
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _lib as L

RECORD_DTYPE = np.dtype([
    ("pid", "<u8"), ("pos", "<f8", (3,)), ("dir", "<f8", (3,)), ("j", "<i4"),
    ("status", "<i4"), ("weight", "<f8"), ("n_cross", "<u8"), ("n_scat", "<u8"),
    ("n_abs", "<u8"), ("n_mrw", "<u8"), ("n_lucy", "<u8"), ("min_margin", "<f8"),
])
assert RECORD_DTYPE.itemsize == C.sizeof(L.PacketRecord)


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _stream(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return None
    return C.c_void_p(stream)


def run_opts(mode="bw_ticket", n_iter=3, epoch_packets=4096, n_total=0, lucy_tau=1e-2,
             mrw_tau=0.0, mrw_gamma=2.0, max_interactions=10_000_000, sed_theta_bins=10,
             record=False, blocks_per_cu=0, queue_depth=0, walk_blocks_per_cu=0,
             tau_mode="flight", src_strata=0, pah_nc=0.0, pah_tcool=0.0, sh_order=0):
    modes = {"frozen": L.FROZEN, "bw_epoch": L.BW_EPOCH, "bw_ticket": L.BW_TICKET}
    o = L.RunOpts()
    o.mode = modes[mode] if isinstance(mode, str) else int(mode)
    o.n_iter, o.epoch_packets, o.n_total = n_iter, epoch_packets, n_total
    o.lucy_tau, o.mrw_tau, o.mrw_gamma = lucy_tau, mrw_tau, mrw_gamma
    o.max_interactions, o.sed_theta_bins, o.record = max_interactions, sed_theta_bins, int(record)
    o.blocks_per_cu, o.queue_depth, o.walk_blocks_per_cu = blocks_per_cu, queue_depth, walk_blocks_per_cu
    taus = {"flight": 0, "per_cell": 1}
    o.tau_mode = taus[tau_mode] if isinstance(tau_mode, str) else int(tau_mode)
    o.src_strata = src_strata
    o.pah_nc, o.pah_tcool = pah_nc, pah_tcool
    o.sh_order = sh_order
    return o


class Context:
    """One model on one GPU: grid, dust, sources, views and tallies."""

    def __init__(self, device: int = 0, precision: str = "fp64"):
        self.lib = L.lib()
        self.fp64 = precision == "fp64"
        h = C.c_void_p()
        L.check(self.lib.mcrt_create(C.byref(h), device, L.FP64 if self.fp64 else L.FP32))
        self.h = h
        self.device = device
        self.nx = self.ny = self.nz = 0
        self.ns = self.nl = 0
        self.nview = self.nimg = 0
        self.nsub = 0
        self.ntheta = 10

    def close(self):
        if self.h:
            self.lib.mcrt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        L.check(st, self.h)

    @property
    def ncells(self):
        """Leaf cells: cubes plus the sub-cubes of divided cubes."""
        return self.nx * self.ny * self.nz + self.nsub

    @property
    def real_dtype(self):
        return np.float64 if self.fp64 else np.float32

    # ------------------------------------------------------------ set-up
    def set_grid(self, rho, origin, dcell):
        self.nsub = 0
        if hasattr(rho, "data_ptr"):  # torch tensor (host or device)
            nz, ny, nx = rho.shape
            dev = rho.is_cuda
            dt = L.FP64 if str(rho.dtype) == "torch.float64" else L.FP32
            ptr = C.c_void_p(rho.data_ptr())
            mem = L.DEVICE if dev else L.HOST
        else:
            a = np.ascontiguousarray(rho)
            if a.dtype not in (np.float64, np.float32):
                a = a.astype(np.float64)
            nz, ny, nx = a.shape
            dt = L.FP64 if a.dtype == np.float64 else L.FP32
            ptr = C.c_void_p(a.ctypes.data)
            mem = L.HOST
            self._keep = a
        o = _f64(origin)
        self._chk(self.lib.mcrt_set_grid(self.h, nx, ny, nz, _dptr(o), float(dcell), ptr, dt, mem))
        self.nx, self.ny, self.nz = nx, ny, nz

    def voxelize_torus(self, n, origin, dcell, geo):
        self.nsub = 0
        o = _f64(origin)
        cen = _f64(geo["centres"])
        self._chk(self.lib.mcrt_voxelize_torus(
            self.h, n[0], n[1], n[2], _dptr(o), float(dcell), cen.shape[0], _dptr(cen),
            geo["r_clump"], geo["rho_clump"], geo["rho_inter"], geo["r_in"], geo["r_out"],
            geo["sin_theta1"]))
        self.nx, self.ny, self.nz = n

    def voxelize_shell(self, n, origin, dcell, geo):
        self.nsub = 0
        o = _f64(origin)
        self._chk(self.lib.mcrt_voxelize_shell(self.h, n[0], n[1], n[2], _dptr(o), float(dcell),
                                               geo["rho0"], geo["r_in"], geo["r_out"],
                                               float(geo.get("power", 2.0))))
        self.nx, self.ny, self.nz = n

    def set_dust(self, lam_um, mass_frac, kabs, ksca, g, pah_species=-1, pah_emis=None,
                 pah_edges=None):
        lam, fr = _f64(lam_um), _f64(mass_frac)
        ka, ks, gg = _f64(kabs), _f64(ksca), _f64(g)
        pe, ped = _f64(pah_emis), _f64(pah_edges)
        rows = 0 if pe is None else pe.shape[0]
        self._chk(self.lib.mcrt_set_dust(self.h, lam.size, _dptr(lam), fr.size, _dptr(fr),
                                         _dptr(ka), _dptr(ks), _dptr(gg), pah_species, rows,
                                         _dptr(pe), _dptr(ped)))
        self.nl, self.ns = lam.size, fr.size

    def set_sources(self, pos, lum, shape=None, t_bb=None):
        p, l = _f64(pos), _f64(lum)
        sh, tb = _f64(shape), _f64(t_bb)
        self._chk(self.lib.mcrt_set_sources(self.h, l.size, _dptr(p), _dptr(l), _dptr(sh),
                                            _dptr(tb)))

    def set_views(self, views_deg, img_idx, distance):
        v = _f64(views_deg) if views_deg is not None else np.zeros((0, 2))
        idx = np.ascontiguousarray(img_idx if img_idx is not None else [], dtype=np.int32)
        self._chk(self.lib.mcrt_set_views(self.h, v.shape[0], _dptr(v), idx.size,
                                          idx.ctypes.data_as(C.POINTER(C.c_int32)),
                                          float(distance)))
        self.nview, self.nimg = v.shape[0], idx.size

    def from_inputs(self, mi, views=None, img_idx=None, distance=1.0):
        """Configure grid, dust and sources from a mcrt_inputs.ModelInputs."""
        geo = mi.geometry or {}
        if mi.rho is not None:
            self.set_grid(mi.rho, mi.origin, mi.dcell)
        elif geo.get("kind") == "torus":
            self.voxelize_torus((mi.nx, mi.ny, mi.nz), mi.origin, mi.dcell, geo)
        elif geo.get("kind") == "shell":
            self.voxelize_shell((mi.nx, mi.ny, mi.nz), mi.origin, mi.dcell, geo)
        else:
            raise ValueError("model has neither rho nor a voxelizable geometry")
        self.set_dust(mi.lam_um, mi.mass_frac, mi.kabs, mi.ksca, mi.g, mi.pah_species,
                      mi.pah_emis, mi.pah_edges)
        if getattr(mi, "ref", None) is not None:
            self.set_refinement(mi.ref, mi.rho_sub)
        self.set_sources(mi.src_pos, mi.src_lum, mi.src_shape, mi.src_tbb)
        if views is not None:
            self.set_views(views, img_idx, distance)
        return self

    def set_refinement(self, ref, rho_sub):
        """Divide cube c into ref[c]^3 sub-cubes (ref >= 2) with densities
        rho_sub, cube by cube in linear cube order, x fastest inside a cube."""
        r = None if ref is None else np.ascontiguousarray(ref, dtype=np.uint8).ravel()
        rs = _f64(rho_sub) if rho_sub is not None else np.zeros(0)
        self._chk(self.lib.mcrt_set_refinement(
            self.h, None if r is None else r.ctypes.data_as(C.POINTER(C.c_uint8)),
            C.c_void_p(rs.ctypes.data) if rs.size else None, rs.size, L.FP64))
        self.nsub = int(rs.size)

    # -------------------------------------------------------------- runs
    def reset(self, stream=None):
        self._chk(self.lib.mcrt_reset(self.h, _stream(stream)))

    def init_temperatures(self, stream=None):
        self._chk(self.lib.mcrt_init_temperatures(self.h, _stream(stream)))

    def set_temperatures(self, T):
        a = _f64(T)
        self._chk(self.lib.mcrt_set_temperatures(self.h, C.c_void_p(a.ctypes.data), L.HOST, None))

    def set_scattering(self, ssca):
        a = _f64(ssca)
        self._chk(self.lib.mcrt_set_scattering(self.h, C.c_void_p(a.ctypes.data), L.HOST, None))

    def run_packets(self, first=0, n=0, seed=0, stream=None, **opts):
        o = run_opts(**opts)
        self.ntheta = o.sed_theta_bins
        st = L.RunStats()
        self._chk(self.lib.mcrt_run_packets(self.h, first, n, seed, C.byref(o), C.byref(st),
                                            _stream(stream)))
        return {n_: getattr(st, n_) for n_ in L.STAT_NAMES + ["kernel_ms"]}

    def run_pah(self, seed=0, stream=None, **opts):
        o = run_opts(**opts)
        st = L.RunStats()
        self._chk(self.lib.mcrt_run_pah(self.h, seed, C.byref(o), C.byref(st), _stream(stream)))
        return {n_: getattr(st, n_) for n_ in L.STAT_NAMES + ["kernel_ms"]}

    # ----------------------------------------------------------- outputs
    def finalize_temperatures(self, stream=None):
        """Eq. 4 on the device into the context's temperature field (no copy)."""
        self._chk(self.lib.mcrt_temperatures(self.h, None, None, L.DEVICE, _stream(stream)))

    def temperatures(self, with_energy=False):
        T = np.zeros((self.ns, self.ncells))
        E = np.zeros((self.ns, self.ncells)) if with_energy else None
        self._chk(self.lib.mcrt_temperatures(self.h, C.c_void_p(T.ctypes.data),
                                             C.c_void_p(E.ctypes.data) if E is not None else None,
                                             L.HOST, None))
        return (T, E) if with_energy else T

    def invert_temperature(self, species, rhs, method=0):
        r = _f64(rhs).ravel()
        T = np.zeros_like(r)
        self._chk(self.lib.mcrt_invert_temperature(self.h, species, r.size, C.c_void_p(r.ctypes.data),
                                                   C.c_void_p(T.ctypes.data), method))
        return T

    def current_temperatures(self):
        T = np.zeros((self.ns, self.ncells))
        self._chk(self.lib.mcrt_get_temperatures(self.h, C.c_void_p(T.ctypes.data), L.HOST, None))
        return T

    def density(self):
        r = np.zeros(self.ncells, dtype=self.real_dtype)
        self._chk(self.lib.mcrt_density(self.h, C.c_void_p(r.ctypes.data), L.HOST, None))
        return r

    def tallies(self):
        k = np.zeros((self.ns, self.ncells), dtype=np.uint64)
        ep = np.zeros((self.ns, self.ncells))
        kp = np.zeros(self.ncells, dtype=np.uint32)
        self._chk(self.lib.mcrt_tallies(self.h, C.c_void_p(k.ctypes.data),
                                        C.c_void_p(ep.ctypes.data), C.c_void_p(kp.ctypes.data),
                                        L.HOST, None))
        return k, ep, kp

    def sed(self):
        f = np.zeros((self.ntheta, self.nl))
        c = np.zeros((self.ntheta, self.nl), dtype=np.uint64)
        self._chk(self.lib.mcrt_sed(self.h, C.c_void_p(f.ctypes.data), C.c_void_p(c.ctypes.data),
                                    L.HOST, None))
        return f, c

    def scattering(self):
        s = np.zeros((self.nview, self.nimg, self.ncells))
        self._chk(self.lib.mcrt_scattering(self.h, C.c_void_p(s.ctypes.data), L.HOST, None))
        return s

    def records(self, n):
        r = np.zeros(n, dtype=RECORD_DTYPE)
        self._chk(self.lib.mcrt_packet_records(self.h, C.c_void_p(r.ctypes.data), n, L.HOST))
        return r

    def raytrace(self, npx, npy, rho_rt=None, stream=None):
        """Images [view][img][npy][npx] (numpy) and SED [view][img]."""
        img = np.zeros((self.nview, self.nimg, npy, npx), dtype=self.real_dtype)
        sed = np.zeros((self.nview, self.nimg))
        rr = None if rho_rt is None else C.c_void_p(rho_rt.data_ptr())
        self._chk(self.lib.mcrt_raytrace_image(self.h, npx, npy, rr, C.c_void_p(img.ctypes.data),
                                               C.c_void_p(sed.ctypes.data), L.HOST,
                                               _stream(stream)))
        return img, sed

    def raytrace_adjoint(self, npx, npy, w_img=None, w_sed=None, rho_rt=None, stream=None):
        g = np.zeros(self.ncells, dtype=self.real_dtype)
        wi = None if w_img is None else np.ascontiguousarray(w_img, dtype=self.real_dtype)
        ws = _f64(w_sed)
        rr = None if rho_rt is None else C.c_void_p(rho_rt.data_ptr())
        self._chk(self.lib.mcrt_raytrace_adjoint(
            self.h, npx, npy, rr, C.c_void_p(wi.ctypes.data) if wi is not None else None,
            C.c_void_p(ws.ctypes.data) if ws is not None else None, C.c_void_p(g.ctypes.data),
            L.HOST, _stream(stream)))
        return g

    # device-resident variants (torch tensors, current stream)
    def raytrace_device(self, npx, npy, rho_rt=None, img=None, sed=None):
        import torch
        dt = torch.float64 if self.fp64 else torch.float32
        dev = torch.device("cuda", self.device)
        if img is None:
            img = torch.empty((self.nview, self.nimg, npy, npx), dtype=dt, device=dev)
        if sed is None:
            sed = torch.empty((self.nview, self.nimg), dtype=torch.float64, device=dev)
        rr = None if rho_rt is None else C.c_void_p(rho_rt.data_ptr())
        self._chk(self.lib.mcrt_raytrace_image(self.h, npx, npy, rr, C.c_void_p(img.data_ptr()),
                                               C.c_void_p(sed.data_ptr()), L.DEVICE,
                                               _stream(None)))
        return img, sed

    def set_scattering_law(self, law):
        """'hg' (Henyey-Greenstein) or 'gfactor' (isotropic, kappa_sca (1 - g))."""
        laws = {"hg": 0, "gfactor": 1}
        self._chk(self.lib.mcrt_set_scattering_law(self.h, laws[law] if isinstance(law, str)
                                                   else int(law)))

    def set_scattered_light(self, source):
        """'peeloff' (per-view sums of the run) or 'moments' (any view)."""
        srcs = {"peeloff": 0, "moments": 1}
        self._chk(self.lib.mcrt_set_scattered_light(self.h, srcs[source] if isinstance(source, str)
                                                    else int(source)))

    def scattering_moments(self):
        """Moments [img][order^2][cells] in erg/s (None when there are none)."""
        order = C.c_int()
        self._chk(self.lib.mcrt_scattering_moments(self.h, None, C.byref(order), L.HOST, None))
        if order.value == 0:
            return None
        out = np.zeros((self.nimg, order.value ** 2, self.ncells))
        self._chk(self.lib.mcrt_scattering_moments(self.h, C.c_void_p(out.ctypes.data), None,
                                                   L.HOST, None))
        return out

    def set_raytrace_mode(self, mode):
        """'ext' (chord form) or 'abs_literal' (Eqs. 13-14 as printed)."""
        modes = {"ext": 0, "abs_literal": 1}
        self._chk(self.lib.mcrt_set_raytrace_mode(self.h, modes[mode] if isinstance(mode, str)
                                                  else int(mode)))

    def raytrace_noalloc(self, npx, npy, img, sed=None, rho_rt=None):
        """mcrt_raytrace_image_noalloc into caller-owned device tensors."""
        rr = None if rho_rt is None else C.c_void_p(rho_rt.data_ptr())
        self._chk(self.lib.mcrt_raytrace_image_noalloc(
            self.h, npx, npy, rr, C.c_void_p(img.data_ptr()),
            None if sed is None else C.c_void_p(sed.data_ptr()), _stream(None)))
        return img, sed

    def raytrace_adjoint_device(self, npx, npy, w_img=None, w_sed=None, rho_rt=None, out=None):
        import torch
        dt = torch.float64 if self.fp64 else torch.float32
        if out is None:
            out = torch.empty(self.ncells, dtype=dt, device=torch.device("cuda", self.device))
        self._chk(self.lib.mcrt_raytrace_adjoint(
            self.h, npx, npy, None if rho_rt is None else C.c_void_p(rho_rt.data_ptr()),
            None if w_img is None else C.c_void_p(w_img.data_ptr()),
            None if w_sed is None else C.c_void_p(w_sed.data_ptr()),
            C.c_void_p(out.data_ptr()), L.DEVICE, _stream(None)))
        return out

    def timings(self):
        t = (C.c_double(), C.c_double(), C.c_double())
        self._chk(self.lib.mcrt_last_timings(self.h, C.byref(t[0]), C.byref(t[1]), C.byref(t[2])))
        b = C.c_double()
        self._chk(self.lib.mcrt_last_source_build_ms(self.h, C.byref(b)))
        return {"transport_ms": t[0].value, "rt_fwd_ms": t[1].value, "rt_adj_ms": t[2].value,
                "build_S_ms": b.value}

    def sample_reemission(self, species, T, n, seed=0, mode="bw_ticket"):
        """Histogram [n_lambda] of n re-emission bins at temperature T (see
        mcrt_sample_reemission)."""
        modes = {"frozen": L.FROZEN, "bw_epoch": L.BW_EPOCH, "bw_ticket": L.BW_TICKET}
        out = np.zeros(self.nl, dtype=np.uint64)
        self._chk(self.lib.mcrt_sample_reemission(
            self.h, int(species), modes[mode] if isinstance(mode, str) else int(mode), float(T),
            int(n), int(seed), out.ctypes.data_as(C.POINTER(C.c_uint64))))
        return out

    def phase_timings(self):
        """Emission, walk and interaction kernel time (ms) of the last run, and its rounds."""
        t = (C.c_double(), C.c_double(), C.c_double())
        r = C.c_uint64()
        self._chk(self.lib.mcrt_phase_timings(self.h, C.byref(t[0]), C.byref(t[1]), C.byref(t[2]),
                                              C.byref(r)))
        return {"emit_ms": t[0].value, "walk_ms": t[1].value, "interact_ms": t[2].value,
                "rounds": r.value}


def run_batch(contexts, n_packets, seeds, stream=None, **opts):
    """Wavefront rounds over many contexts in one replayed HIP graph (see mcrt_run_batch)."""
    lib = L.lib()
    n = len(contexts)
    arr = (C.c_void_p * n)(*[c.h.value for c in contexts])
    npk = (C.c_uint64 * n)(*[int(x) for x in n_packets])
    sd = (C.c_uint64 * n)(*[int(x) for x in seeds])
    o = run_opts(**opts)
    st = (L.RunStats * n)()
    L.check(lib.mcrt_run_batch(arr, n, npk, sd, C.byref(o), st, _stream(stream)), contexts[0].h)
    for c in contexts:
        c.ntheta = o.sed_theta_bins
    return [{n_: getattr(s, n_) for n_ in L.STAT_NAMES + ["kernel_ms"]} for s in st]
