"""ctypes binding of libpyronn_mi.so (the C ABI in include/pyronn_mi.h).

Argument marshalling only: every operator runs in the HIP kernels of the
library.  Importing this module loads the library and raises ImportError if
it has not been built; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpyronn_mi.so")

PN_F32, PN_BF16, PN_F16 = 0, 1, 2
PN_PARALLEL, PN_FAN, PN_CONE = 0, 1, 2
PN_OK, PN_EINVAL, PN_EDTYPE, PN_EGEOM, PN_EHIP, PN_ENOMEM = 0, -1, -2, -3, -4, -5
ERROR_NAMES = {
    PN_EINVAL: "PN_EINVAL",
    PN_EDTYPE: "PN_EDTYPE",
    PN_EGEOM: "PN_EGEOM",
    PN_EHIP: "PN_EHIP",
    PN_ENOMEM: "PN_ENOMEM",
}

# every symbol the header declares
EXPORTS = (
    "pn_forward",
    "pn_forward_sampled",
    "pn_adjoint",
    "pn_adjoint_noalloc",
    "pn_backproject",
    "pn_backproject_sampled",
    "pn_splat",
    "pn_forward_batched",
    "pn_adjoint_batched",
    "pn_backproject_batched",
    "pn_batch_create",
    "pn_batch_run",
    "pn_batch_destroy",
    "pn_filter",
    "pn_gaussian_noise",
    "pn_detector_jitter",
    "pn_gantry_blur",
    "pn_ring_artifacts",
    "pn_check_geometry",
    "pn_cone_matrices",
    "pn_fan_matrices",
    "pn_parallel2d_matrices",
    "pn_parallel3d_matrices",
    "pn_last_error",
    "pn_release_caches",
    "pn_version",
)


class PnGeometry(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("beam", ctypes.c_int32),
        ("vol_shape", ctypes.c_int64 * 3),
        ("vol_spacing", ctypes.c_double * 3),
        ("vol_origin", ctypes.c_double * 3),
        ("det_shape", ctypes.c_int64 * 2),
        ("det_spacing", ctypes.c_double * 2),
        ("sid", ctypes.c_double),
        ("sdd", ctypes.c_double),
        ("n_views", ctypes.c_int64),
        ("proj", ctypes.POINTER(ctypes.c_double)),
    ]


class PnProblem(ctypes.Structure):
    _fields_ = [("geom", PnGeometry), ("in_", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class PnError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__(f"{where}: {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python paper_2511_08427_amd/csrc/build.py or __graft_entry__.build())"
        )
    lib = ctypes.CDLL(LIB_PATH)
    gp = ctypes.POINTER(PnGeometry)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    dp = ctypes.POINTER(ctypes.c_double)
    for name in ("pn_forward", "pn_adjoint", "pn_adjoint_noalloc", "pn_backproject", "pn_splat"):
        f = getattr(lib, name)
        f.argtypes = [gp, i64, vp, vp, i32, i32, vp]
        f.restype = ctypes.c_int
    for name in ("pn_forward_batched", "pn_adjoint_batched", "pn_backproject_batched"):
        f = getattr(lib, name)
        f.argtypes = [ctypes.POINTER(PnProblem), i32, i32, i32, vp]
        f.restype = ctypes.c_int
    lib.pn_forward_sampled.argtypes = [gp, i64, vp, vp, i32, i32, i32, i32, vp]
    lib.pn_forward_sampled.restype = ctypes.c_int
    lib.pn_backproject_sampled.argtypes = [gp, i64, vp, vp, i32, i32, i32, i32, vp]
    lib.pn_backproject_sampled.restype = ctypes.c_int
    lib.pn_batch_create.argtypes = [i32, ctypes.POINTER(PnProblem), i32, i32, i32, ctypes.POINTER(vp)]
    lib.pn_batch_create.restype = ctypes.c_int
    lib.pn_batch_run.argtypes = [vp, vp]
    lib.pn_batch_run.restype = ctypes.c_int
    lib.pn_batch_destroy.argtypes = [vp]
    lib.pn_batch_destroy.restype = ctypes.c_int
    lib.pn_filter.argtypes = [gp, i64, vp, vp, i32, i32, i32, vp]
    lib.pn_filter.restype = ctypes.c_int
    lib.pn_gaussian_noise.argtypes = [i64, vp, i32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, vp]
    lib.pn_gaussian_noise.restype = ctypes.c_int
    lib.pn_detector_jitter.argtypes = [i64, i32, vp, vp, i32, i32, ctypes.c_uint64, vp]
    lib.pn_detector_jitter.restype = ctypes.c_int
    lib.pn_gantry_blur.argtypes = [i64, i32, i32, i32, vp, vp, i32, ctypes.c_double, ctypes.c_double, i32, vp]
    lib.pn_gantry_blur.restype = ctypes.c_int
    lib.pn_ring_artifacts.argtypes = [i64, i32, i32, i32, vp, i32, ctypes.POINTER(ctypes.c_int32), i32,
                                      ctypes.c_double, i32, i32, vp]
    lib.pn_ring_artifacts.restype = ctypes.c_int
    lib.pn_check_geometry.argtypes = [gp]
    lib.pn_check_geometry.restype = ctypes.c_int
    lib.pn_cone_matrices.argtypes = [i64, dp, dp, dp, dp, i64, i64, dp]
    lib.pn_fan_matrices.argtypes = [i64, dp, dp, dp, i64, dp]
    lib.pn_parallel2d_matrices.argtypes = [i64, dp, dp, dp, i64, dp]
    lib.pn_parallel3d_matrices.argtypes = [i64, dp, dp, dp, dp, i64, i64, dp]
    for name in ("pn_cone_matrices", "pn_fan_matrices", "pn_parallel2d_matrices", "pn_parallel3d_matrices",
                 "pn_release_caches"):
        getattr(lib, name).restype = ctypes.c_int
    lib.pn_last_error.restype = ctypes.c_char_p
    lib.pn_version.restype = ctypes.c_char_p
    return lib


lib = _load()


def last_error() -> str:
    return lib.pn_last_error().decode()


def check(rc, where):
    if rc != PN_OK:
        raise PnError(rc, where, last_error())


def dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
