"""ctypes binding of libssf (include/ssf.h): argument marshalling only.

Every function here forwards to the C ABI of the same name; all arithmetic of
the split-step path runs in the HIP kernels of libssf.so.  The library is
loaded from this package directory; if it is missing the import fails with
an error that says how to build it (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SSF_LIBRARY may point at another build of the same library (e.g. a tile variant)
LIB_PATH = os.environ.get("SSF_LIBRARY") or os.path.join(_HERE, "libssf.so")

SSF_OK = 0
SSF_E_INVALID = -1
SSF_E_UNSUPPORTED = -2
SSF_E_NOMEM = -3
SSF_E_NODEVICE = -4
SSF_E_DEVICE = -5
SSF_E_NONFINITE = -6
SSF_C64 = 1
SSF_C128 = 2
SSF_REAL = 0
SSF_IMAG = 1
SSF_SPLIT_VTV = 0
SSF_SPLIT_TVT = 1
SSF_TILE_VARIANTS = 3
SSF_ARITH_F64 = 0
SSF_ARITH_F32 = 1

EXPORTS = (
    "ssf_supported_length", "ssf_create", "ssf_destroy", "ssf_set_stream",
    "ssf_set_potential_table", "ssf_set_potential_ctap", "ssf_clear_potential",
    "ssf_set_partition", "ssf_set_partition_z", "ssf_set_fusion", "ssf_set_splitting", "ssf_set_timing", "ssf_timing_read",
    "ssf_tune", "ssf_set_tiles", "ssf_get_tiles", "ssf_step", "ssf_fft", "ssf_observables",
    "ssf_obs_read", "ssf_density_xz", "ssf_sync", "ssf_copy", "ssf_step_ckpt", "ssf_step_seq", "ssf_adjoint_init",
    "ssf_adjoint_segment", "ssf_profile_grad", "ssf_batch_create", "ssf_batch_run", "ssf_batch_tune",
    "ssf_batch_info", "ssf_batch_set_stream", "ssf_batch_destroy", "ssf_bspline_basis", "ssf_bspline_eval", "ssf_status_string", "ssf_last_error",
    "ssf_step_noalloc", "ssf_noalloc_scratch_bytes", "ssf_noalloc_scratch_need",
    "ssf_chip_potential", "ssf_batch_create_tables", "ssf_set_arithmetic", "ssf_tune_cached",
)


class ssf_grid_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


class ssf_ctap_desc(ctypes.Structure):
    _fields_ = [("nguides", ctypes.c_int32), ("v0", ctypes.c_double * 3),
                ("sigma", ctypes.c_double * 3), ("xc", ctypes.POINTER(ctypes.c_double))]


class ssf_chip_desc(ctypes.Structure):
    _fields_ = [("nwires", ctypes.c_int32), ("npts", ctypes.POINTER(ctypes.c_int32)),
                ("path", ctypes.POINTER(ctypes.c_double)), ("current", ctypes.POINTER(ctypes.c_double)),
                ("b_bias", ctypes.c_double), ("b_ip", ctypes.c_double), ("length_unit", ctypes.c_double),
                ("mu_over_e0", ctypes.c_double), ("omega_z", ctypes.c_double), ("z_c", ctypes.c_double)]


class ssf_obs(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_double), ("mean", ctypes.c_double * 3),
                ("pop", ctypes.c_double * 3), ("epot", ctypes.c_double),
                ("energy", ctypes.c_double), ("step", ctypes.c_int64),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


OBS_DTYPE = np.dtype([("norm", "f8"), ("mean", "f8", (3,)), ("pop", "f8", (3,)), ("epot", "f8"),
                      ("energy", "f8"), ("step", "i8"), ("flags", "i4"), ("reserved", "i4")])
assert OBS_DTYPE.itemsize == ctypes.sizeof(ssf_obs)


class SSFError(RuntimeError):
    def __init__(self, status, where, detail):
        super().__init__("%s failed: %s (%d): %s" % (where, _status_name(status), status, detail))
        self.status = status


_lib = None


def _status_name(s):
    return {0: "SSF_OK", -1: "SSF_E_INVALID", -2: "SSF_E_UNSUPPORTED", -3: "SSF_E_NOMEM",
            -4: "SSF_E_NODEVICE", -5: "SSF_E_DEVICE", -6: "SSF_E_NONFINITE"}.get(s, "?")


def load():
    """Load libssf.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libssf.so is not built: run `python -m paper_1309_2451_amd.build` "
                          "(or __graft_entry__.build()) first; there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    vp, dp, i32, i64, dbl = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    hp = ctypes.c_void_p
    sig = {
        "ssf_supported_length": ([i32], i32),
        "ssf_create": ([ctypes.POINTER(ssf_grid_desc), i32, vp, ctypes.POINTER(hp)], i32),
        "ssf_destroy": ([hp], i32),
        "ssf_set_stream": ([hp, vp], i32),
        "ssf_set_potential_table": ([hp, vp, i32], i32),
        "ssf_set_potential_ctap": ([hp, ctypes.POINTER(ssf_ctap_desc)], i32),
        "ssf_clear_potential": ([hp], i32),
        "ssf_set_partition": ([hp, dbl, dbl], i32),
        "ssf_set_partition_z": ([hp, dp, dp], i32),
        "ssf_set_fusion": ([hp, i32], i32),
        "ssf_set_splitting": ([hp, i32], i32),
        "ssf_set_arithmetic": ([hp, i32], i32),
        "ssf_set_timing": ([hp, i32], i32),
        "ssf_tune": ([hp, i32, vp, vp], i32),
        "ssf_tune_cached": ([hp, i32, ctypes.c_char_p, vp, vp], i32),
        "ssf_set_tiles": ([hp, vp], i32),
        "ssf_get_tiles": ([hp, vp], i32),
        "ssf_timing_read": ([hp, vp, vp], i32),
        "ssf_step": ([hp, vp, i64, dbl, i32, i64, vp], i32),
        "ssf_step_noalloc": ([hp, vp, i64, dbl, i32, i64, vp], i32),
        "ssf_noalloc_scratch_bytes": ([], i64),
        "ssf_noalloc_scratch_need": ([hp], i64),
        "ssf_fft": ([hp, vp, i32, i32], i32),
        "ssf_observables": ([hp, vp, vp], i32),
        "ssf_obs_read": ([hp, vp, vp, i64], i32),
        "ssf_density_xz": ([hp, vp, vp], i32),
        "ssf_sync": ([hp], i32),
        "ssf_copy": ([hp, vp, vp], i32),
        "ssf_step_ckpt": ([hp, vp, i64, dbl, i64, vp], i32),
        "ssf_step_seq": ([hp, vp, i64, dbl, vp], i32),
        "ssf_adjoint_init": ([hp, vp, vp], i32),
        "ssf_adjoint_segment": ([hp, vp, vp, i64, dbl, vp], i32),
        "ssf_profile_grad": ([hp, vp, i32, vp, i32, vp], i32),
        "ssf_batch_create": ([i32, vp, vp, dp, dp, i32, vp, ctypes.POINTER(hp)], i32),
        "ssf_batch_run": ([hp, vp, i64, dbl, i64, vp], i32),
        "ssf_batch_create_tables": ([i32, vp, vp, dp, dp, i32, vp, ctypes.POINTER(hp)], i32),
        "ssf_chip_potential": ([hp, ctypes.POINTER(ssf_chip_desc), vp], i32),
        "ssf_batch_tune": ([hp, i32], i32),
        "ssf_batch_info": ([hp, ctypes.POINTER(i32), vp], i32),
        "ssf_batch_set_stream": ([hp, vp], i32),
        "ssf_batch_destroy": ([hp], i32),
        "ssf_bspline_basis": ([i32, dbl, dbl, dp, i32, dp], i32),
        "ssf_bspline_eval": ([i32, dbl, dbl, dp, i32, dp, i32, dp], i32),
        "ssf_status_string": ([i32], ctypes.c_char_p),
        "ssf_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def check(status, where):
    if status != SSF_OK:
        detail = load().ssf_last_error().decode(errors="replace")
        raise SSFError(status, where, detail)
    return status


def call(name, *args):
    """Call an ssf_* function and raise SSFError on a negative status."""
    return check(getattr(load(), name)(*args), name)
