"""ctypes binding of libsht.so (the C ABI in include/sht.h).

Argument marshalling only: every step of the transform runs in the HIP
kernels of the library.  Importing this module without the built library
raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsht.so")

SHT_OK = 0
SHT_ERR_INVALID_ARG = -1
SHT_ERR_OOM = -2
SHT_ERR_HIP = -3
SHT_ERR_UNSUPPORTED = -4
SHT_ERR_BAD_HANDLE = -5
SHT_ERR_WORKSPACE = -6

SHT_FP64 = 0
SHT_FP32_MFMA = 1
SHT_BF16X3_MFMA = 2
SHT_F16X2_MFMA = 3
SHT_FLAG_NO_PAIRING = 1

SHT_NOALLOC_SCRATCH_BYTES = 64 << 20
SHT_MAX_LMAX = 16383
SHT_MAX_NPHI = 16384

EXPORTED = [
    "sht_plan", "sht_plan_destroy", "sht_plan_get_info", "sht_plan_workspace_size",
    "sht_plan_get_config", "sht_plan_set_config", "sht_plan_autotune",
    "sht_alm2map", "sht_alm2map_events", "sht_alm2map_adjoint", "sht_alm2delta", "sht_delta2map",
    "sht_map2delta_adjoint", "sht_delta2alm_adjoint", "sht_map2alm", "sht_status_string",
    "sht_version",
    "sht_plan_batch", "sht_batch_destroy", "sht_batch_workspace_size", "sht_alm2map_batch",
    "sht_batch_get_config", "sht_batch_set_config", "sht_batch_autotune",
    "sht_batch_graph_capture", "sht_batch_graph_launch", "sht_alm2map_noalloc",
]


class GeometryDesc(ctypes.Structure):
    _fields_ = [
        ("lmax", ctypes.c_int32),
        ("nm", ctypes.c_int32),
        ("mval", ctypes.POINTER(ctypes.c_int32)),
        ("nrings", ctypes.c_int32),
        ("cth", ctypes.POINTER(ctypes.c_double)),
        ("sth", ctypes.POINTER(ctypes.c_double)),
        ("phi0", ctypes.POINTER(ctypes.c_double)),
        ("nphi", ctypes.POINTER(ctypes.c_int64)),
        ("ringstart", ctypes.POINTER(ctypes.c_int64)),
        ("nmaps", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("npix", ctypes.c_int64),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("nalm", ctypes.c_int64),
        ("npix", ctypes.c_int64),
        ("nrings", ctypes.c_int32),
        ("npairs", ctypes.c_int32),
        ("nm", ctypes.c_int32),
        ("lmax", ctypes.c_int32),
        ("mmax", ctypes.c_int32),
        ("nmaps", ctypes.c_int32),
        ("workspace_bytes", ctypes.c_size_t),
        ("delta_bytes", ctypes.c_size_t),
        ("table_bytes", ctypes.c_size_t),
        ("forward_workspace_bytes", ctypes.c_size_t),
    ]


class ShtError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _status_string(code)
        super().__init__(f"{where}: {msg} ({code})")


_lib = None


def load(path: str | None = None):
    """Load libsht.so; raises if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(
            f"{p} is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
            "(hipcc --offload-arch=gfx950); the transform has no CPU implementation")
    # torch ships its own HIP runtime (same soname as the system one).  Load
    # it first so that libsht.so binds to it: loaded the other way round the
    # process holds two runtimes, and torch's memory and streams are foreign
    # to the library's.
    import torch  # noqa: F401

    L = ctypes.CDLL(p)
    vp = ctypes.c_void_p
    L.sht_plan.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(GeometryDesc)]
    L.sht_plan_destroy.argtypes = [vp]
    L.sht_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    L.sht_plan_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.sht_alm2map.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.sht_alm2map_events.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, vp,
                                     ctypes.POINTER(ctypes.c_void_p)]
    L.sht_alm2map_adjoint.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.sht_alm2map_noalloc.argtypes = [vp, vp, vp, vp]
    L.sht_alm2delta.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.sht_delta2map.argtypes = [vp, vp, vp, vp]
    L.sht_map2delta_adjoint.argtypes = [vp, vp, vp, vp]
    L.sht_delta2alm_adjoint.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.sht_map2alm.argtypes = [vp, vp, vp, vp, ctypes.c_int32, vp, vp, ctypes.c_size_t, vp]
    L.sht_plan_get_config.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.sht_plan_set_config.argtypes = [vp, ctypes.c_int32]
    L.sht_plan_autotune.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, ctypes.c_char_p, vp]
    for fn in ["sht_plan", "sht_plan_destroy", "sht_plan_get_info", "sht_plan_workspace_size",
               "sht_alm2map", "sht_alm2map_events", "sht_alm2map_adjoint", "sht_alm2delta", "sht_delta2map",
               "sht_alm2map_noalloc",
               "sht_map2delta_adjoint", "sht_delta2alm_adjoint", "sht_map2alm",
               "sht_plan_get_config", "sht_plan_set_config", "sht_plan_autotune"]:
        getattr(L, fn).restype = ctypes.c_int
    L.sht_plan_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int32]
    L.sht_batch_destroy.argtypes = [vp]
    L.sht_batch_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.sht_alm2map_batch.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.sht_batch_get_config.argtypes = [vp, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]
    L.sht_batch_set_config.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    L.sht_batch_autotune.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, ctypes.c_char_p, vp]
    L.sht_batch_graph_capture.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.sht_batch_graph_launch.argtypes = [vp, vp]
    for fn in ["sht_plan_batch", "sht_batch_destroy", "sht_batch_workspace_size",
               "sht_alm2map_batch", "sht_batch_get_config", "sht_batch_set_config",
               "sht_batch_autotune", "sht_batch_graph_capture", "sht_batch_graph_launch"]:
        getattr(L, fn).restype = ctypes.c_int
    L.sht_status_string.argtypes = [ctypes.c_int]
    L.sht_status_string.restype = ctypes.c_char_p
    L.sht_version.argtypes = []
    L.sht_version.restype = ctypes.c_char_p
    _lib = L
    return L


def _status_string(code: int) -> str:
    try:
        return load().sht_status_string(int(code)).decode()
    except Exception:  # pragma: no cover
        return "status"


def check(code: int, where: str) -> None:
    if code != SHT_OK:
        raise ShtError(code, where)
