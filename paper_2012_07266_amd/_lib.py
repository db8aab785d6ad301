"""ctypes binding of libmadlens_amd.so (argument marshalling only).

The shared library is built in-tree by `python -m paper_2012_07266_amd.build`
(or `__graft_entry__.build()`).  Loading fails loudly when it is missing:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmadlens_amd.so")

PM_OK, PM_EINVAL, PM_ENOMEM, PM_EDEVICE, PM_ESTATE, PM_ENONFINITE, PM_EAGAIN, PM_ETOOBIG = \
    0, -1, -2, -3, -4, -5, -7, -8
PM_EFULL = -9
PM_NOALLOC_MAX_BYTES = 64 << 20
PM_F32, PM_F64 = 0, 1
PM_MODE_PGD, PM_MODE_TANGENT, PM_MODE_CKPT_FORCE = 1, 2, 4


class PmParams(ctypes.Structure):
    _fields_ = [("np", ctypes.c_int32), ("nm", ctypes.c_int32),
                ("box", ctypes.c_double), ("omega_m", ctypes.c_double),
                ("omega_b", ctypes.c_double), ("h", ctypes.c_double),
                ("n_s", ctypes.c_double), ("sigma8", ctypes.c_double),
                ("t_cmb", ctypes.c_double), ("dtype", ctypes.c_int32),
                ("modes", ctypes.c_uint32)]


class LensParams(ctypes.Structure):
    _fields_ = [("npix", ctypes.c_int32), ("fov_deg", ctypes.c_double),
                ("nsrc", ctypes.c_int32), ("z_src", ctypes.POINTER(ctypes.c_double))]


class PmRequest(ctypes.Structure):
    _fields_ = [("p", PmParams), ("l", LensParams), ("a_start", ctypes.c_double),
                ("a_end", ctypes.c_double), ("nsteps", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class PmSrvStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("running", ctypes.c_int32),
                ("queued", ctypes.c_int32), ("peak_running", ctypes.c_int32),
                ("bytes_in_use", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t),
                ("now", ctypes.c_double)]


# name -> (restype, argtypes); every entry point declared in include/madlens.h
_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
SIGNATURES = {
    "pm_footprint": (ctypes.c_size_t, [ctypes.POINTER(PmParams), ctypes.POINTER(LensParams)]),
    "pm_create": (_I, [ctypes.POINTER(PmParams), ctypes.POINTER(LensParams), _P,
                       ctypes.POINTER(_P)]),
    "pm_destroy": (_I, [_P]),
    "pm_init_ic": (_I, [_P, _P, _D]),
    "pm_init_ic_seed": (_I, [_P, ctypes.c_uint64, _D]),
    "pm_noise": (_I, [_P, ctypes.c_uint64, _P]),
    "pm_reconfigure": (_I, [_P, ctypes.POINTER(PmParams), ctypes.POINTER(LensParams)]),
    "pm_step": (_I, [_P, _D, _D]),
    "pm_run": (_I, [_P, ctypes.POINTER(_D), ctypes.c_int32, _P]),
    "lens_project": (_I, [_P, _D, _D, _P]),
    "pm_set_interpolation": (_I, [_P, ctypes.c_int32]),
    "pm_set_pgd": (_I, [_P, ctypes.c_int32, _D, _D, _D, _D]),
    "pm_set_replica_rotation": (_I, [_P, ctypes.c_int32, ctypes.c_uint64]),
    "pm_get_state": (_I, [_P, _P, _P, ctypes.POINTER(_D)]),
    "pm_set_state": (_I, [_P, _P, _P, _D]),
    "pm_get_force": (_I, [_P, _P, _P, _P]),
    "pm_sync": (_I, [_P]),
    "pm_background": (_I, [_P, _D, ctypes.POINTER(_D)]),
    "lens_project_vjp": (_I, [_P, _D, _D, _P, _P, _P, ctypes.POINTER(_D)]),
    "pm_step_vjp": (_I, [_P, _D, _D, _D, _P, _P, _P, ctypes.POINTER(_D)]),
    "pm_init_ic_vjp": (_I, [_P, _D, _P, _P, _P, ctypes.POINTER(_D)]),
    "pm_checkpoint_bytes": (ctypes.c_size_t, [_P]),
    "pm_checkpoint_save": (_I, [_P, _P]),
    "pm_checkpoint_load": (_I, [_P, _P, _D]),
    "pm_vjp_cosmo_read": (_I, [_P, ctypes.POINTER(_D)]),
    "pm_init_ic_jvp": (_I, [_P, _P, _D, _D]),
    "pm_set_tangent": (_I, [_P, _P, _P, _D]),
    "pm_get_tangent": (_I, [_P, _P, _P, _P]),
    "pm_step_jvp": (_I, [_P, _D, _D]),
    "lens_project_jvp": (_I, [_P, _D, _D, _P]),
    "pm_profile": (_I, [_P, _I]),
    "pm_profile_only": (_I, [_P, ctypes.c_char_p]),
    "pm_profile_read": (_I, [_P, _I, ctypes.c_char_p, ctypes.POINTER(_D),
                             ctypes.POINTER(ctypes.c_long), ctypes.POINTER(_I)]),
    "pm_srv_create": (_I, [ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(_P)]),
    "pm_srv_create_ex": (_I, [ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                              ctypes.POINTER(_P)]),
    "pm_srv_submit": (_I, [_P, ctypes.POINTER(PmRequest), ctypes.POINTER(ctypes.c_int64)]),
    "pm_srv_wait": (_I, [_P, ctypes.c_int64, _D]),
    "pm_srv_result": (_I, [_P, ctypes.c_int64, _P, ctypes.POINTER(_D)]),
    "pm_srv_stats_get": (_I, [_P, ctypes.POINTER(PmSrvStats)]),
    "pm_srv_destroy": (_I, [_P]),
    "pm_batch_create": (_I, [ctypes.POINTER(PmParams), ctypes.POINTER(LensParams), ctypes.c_int32,
                             ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    "pm_batch_attach": (_I, [_P, _P, ctypes.POINTER(_D), ctypes.c_int32,
                             ctypes.POINTER(ctypes.c_int32)]),
    "pm_batch_lens": (_I, [_P, _P, _P]),
    "pm_batch_step": (_I, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "pm_batch_detach": (_I, [_P, _P]),
    "pm_batch_destroy": (_I, [_P]),
    "pm_run_noalloc": (_I, [ctypes.POINTER(PmParams), ctypes.POINTER(LensParams), _P, _P,
                            ctypes.POINTER(_D), ctypes.c_int32, _P]),
    "pm_strerror": (ctypes.c_char_p, [_I]),
}

_lib = None


def lib():
    """Load the library once; raise if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2012_07266_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class MadlensError(RuntimeError):
    def __init__(self, code, what):
        msg = lib().pm_strerror(code).decode()
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


def check(code, what):
    if code != PM_OK:
        raise MadlensError(code, what)
    return code
