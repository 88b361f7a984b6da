"""ctypes declarations of libmcrt.so (the C ABI in include/mcrt.h).

Loading fails loudly when the library has not been built: there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcrt.so")

OK, EINVAL, ENOMEM, ESTATE, EDEVICE = 0, -1, -2, -3, -4
HOST, DEVICE = 0, 1
FP64, FP32 = 0, 1
FROZEN, BW_EPOCH, BW_TICKET = 0, 1, 2
ESCAPED, KILLED, PAH_STOP = 1, 2, 3

STAT_NAMES = ["packets", "escaped", "killed", "pah_stopped", "crossings", "scatters",
              "absorptions", "mrw_steps", "lucy_deposits", "clamped_T"]


class RunOpts(C.Structure):
    _fields_ = [
        ("mode", C.c_int32), ("n_iter", C.c_int32), ("epoch_packets", C.c_uint64),
        ("n_total", C.c_uint64), ("lucy_tau", C.c_double), ("mrw_tau", C.c_double),
        ("mrw_gamma", C.c_double), ("max_interactions", C.c_uint64),
        ("sed_theta_bins", C.c_int32), ("record", C.c_int32), ("blocks_per_cu", C.c_int32),
        ("queue_depth", C.c_int32), ("walk_blocks_per_cu", C.c_int32),
        ("tau_mode", C.c_int32), ("src_strata", C.c_uint64), ("pah_nc", C.c_double),
        ("pah_tcool", C.c_double), ("sh_order", C.c_int32), ("pad_", C.c_int32),
    ]


class RunStats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in STAT_NAMES] + [("kernel_ms", C.c_double)]


class PacketRecord(C.Structure):
    _fields_ = [
        ("pid", C.c_uint64), ("pos", C.c_double * 3), ("dir", C.c_double * 3),
        ("j", C.c_int32), ("status", C.c_int32), ("weight", C.c_double),
        ("n_cross", C.c_uint64), ("n_scat", C.c_uint64), ("n_abs", C.c_uint64),
        ("n_mrw", C.c_uint64), ("n_lucy", C.c_uint64), ("min_margin", C.c_double),
    ]


_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
_ctxp = C.c_void_p

# name -> (restype, argtypes)
SIGNATURES = {
    "mcrt_create": (C.c_int, [C.POINTER(_ctxp), C.c_int, C.c_int]),
    "mcrt_destroy": (None, [_ctxp]),
    "mcrt_last_error": (C.c_char_p, [_ctxp]),
    "mcrt_set_grid": (C.c_int, [_ctxp, C.c_int, C.c_int, C.c_int, _dp, C.c_double, _vp, C.c_int,
                                C.c_int]),
    "mcrt_voxelize_torus": (C.c_int, [_ctxp, C.c_int, C.c_int, C.c_int, _dp, C.c_double, C.c_int,
                                      _dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                      C.c_double, C.c_double]),
    "mcrt_voxelize_shell": (C.c_int, [_ctxp, C.c_int, C.c_int, C.c_int, _dp, C.c_double,
                                      C.c_double, C.c_double, C.c_double, C.c_double]),
    "mcrt_set_dust": (C.c_int, [_ctxp, C.c_int, _dp, C.c_int, _dp, _dp, _dp, _dp, C.c_int,
                                C.c_int, _dp, _dp]),
    "mcrt_set_sources": (C.c_int, [_ctxp, C.c_int, _dp, _dp, _dp, _dp]),
    "mcrt_set_views": (C.c_int, [_ctxp, C.c_int, _dp, C.c_int, C.POINTER(C.c_int32), C.c_double]),
    "mcrt_reset": (C.c_int, [_ctxp, _vp]),
    "mcrt_init_temperatures": (C.c_int, [_ctxp, _vp]),
    "mcrt_set_temperatures": (C.c_int, [_ctxp, _vp, C.c_int, _vp]),
    "mcrt_set_scattering": (C.c_int, [_ctxp, _vp, C.c_int, _vp]),
    "mcrt_run_packets": (C.c_int, [_ctxp, C.c_uint64, C.c_uint64, C.c_uint64,
                                   C.POINTER(RunOpts), C.POINTER(RunStats), _vp]),
    "mcrt_run_pah": (C.c_int, [_ctxp, C.c_uint64, C.POINTER(RunOpts), C.POINTER(RunStats), _vp]),
    "mcrt_temperatures": (C.c_int, [_ctxp, _vp, _vp, C.c_int, _vp]),
    "mcrt_tallies": (C.c_int, [_ctxp, _vp, _vp, _vp, C.c_int, _vp]),
    "mcrt_get_temperatures": (C.c_int, [_ctxp, _vp, C.c_int, _vp]),
    "mcrt_invert_temperature": (C.c_int, [_ctxp, C.c_int, C.c_uint64, _vp, _vp, C.c_int]),
    "mcrt_density": (C.c_int, [_ctxp, _vp, C.c_int, _vp]),
    "mcrt_sed": (C.c_int, [_ctxp, _vp, _vp, C.c_int, _vp]),
    "mcrt_scattering": (C.c_int, [_ctxp, _vp, C.c_int, _vp]),
    "mcrt_packet_records": (C.c_int, [_ctxp, _vp, C.c_uint64, C.c_int]),
    "mcrt_raytrace_image": (C.c_int, [_ctxp, C.c_int, C.c_int, _vp, _vp, _vp, C.c_int, _vp]),
    "mcrt_set_raytrace_mode": (C.c_int, [_ctxp, C.c_int]),
    "mcrt_set_refinement": (C.c_int, [_ctxp, C.POINTER(C.c_uint8), _vp, C.c_uint64, C.c_int]),
    "mcrt_set_scattering_law": (C.c_int, [_ctxp, C.c_int]),
    "mcrt_set_scattered_light": (C.c_int, [_ctxp, C.c_int]),
    "mcrt_scattering_moments": (C.c_int, [_ctxp, _vp, C.POINTER(C.c_int), C.c_int, _vp]),
    "mcrt_raytrace_image_noalloc": (C.c_int, [_ctxp, C.c_int, C.c_int, _vp, _vp, _vp, _vp]),
    "mcrt_raytrace_adjoint": (C.c_int, [_ctxp, C.c_int, C.c_int, _vp, _vp, _vp, _vp, C.c_int,
                                        _vp]),
    "mcrt_run_batch": (C.c_int, [C.POINTER(_ctxp), C.c_int, C.POINTER(C.c_uint64),
                                 C.POINTER(C.c_uint64), C.POINTER(RunOpts), C.POINTER(RunStats),
                                 _vp]),
    "mcrt_last_timings": (C.c_int, [_ctxp, _dp, _dp, _dp]),
    "mcrt_last_source_build_ms": (C.c_int, [_ctxp, _dp]),
    "mcrt_phase_timings": (C.c_int, [_ctxp, _dp, _dp, _dp, C.POINTER(C.c_uint64)]),
    "mcrt_sample_reemission": (C.c_int, [_ctxp, C.c_int, C.c_int, C.c_double, C.c_uint64,
                                         C.c_uint64, C.POINTER(C.c_uint64)]),
}

_lib = None


class McrtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mcrt status {status}: {msg}")
        self.status = status


def lib():
    """The loaded libmcrt.so with argument types declared (raises if missing)."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime with the same soname as the system
        # one. Loading torch first makes libmcrt bind to that already-loaded
        # runtime, so device pointers and streams from torch and the library's
        # kernels share one runtime in the process.
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status, ctx=None):
    if status != OK:
        msg = lib().mcrt_last_error(ctx)
        raise McrtError(status, msg.decode() if msg else "")
