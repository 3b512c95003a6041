"""ctypes binding of the C ABI in include/nursd.h (argument marshalling only).

The shared library libnursd.so is built in-tree by
paper_2501_05244_amd/build.py.  Loading fails loudly if it is missing: there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_size_t, c_void_p

# NURSD_LIB names another build of the same library (e.g. a compile-time variant)
LIB_PATH = os.environ.get("NURSD_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnursd.so")

NURSD_OK = 0
ERRORS = {
    -1: "NURSD_ERR_ARG",
    -2: "NURSD_ERR_GEOMETRY",
    -3: "NURSD_ERR_UNSUPPORTED_SIZE",
    -4: "NURSD_ERR_WORKSPACE",
    -5: "NURSD_ERR_HIP",
    -6: "NURSD_ERR_UNIMPLEMENTED",
}
MODE_GRID, MODE_POINTS, MODE_SRSD, MODE_SRSD_POINTS, MODE_GRID3D = 0, 1, 2, 3, 4
STAGES = ["phasor", "spread", "fine_y", "kernel_rows", "propagate_cols", "propagate_rows", "chirp_rows",
          "relay_grid", "type2", "adjoint", "video", "nursd3d"]
NUM_STAGES = 16


class Wavelet(ctypes.Structure):
    _fields_ = [
        ("lambda_c", c_double), ("sigma_rel", c_double), ("n_freq", c_int32), ("n_time", c_int32),
        ("dt", c_double), ("t0", c_double), ("bins", POINTER(c_int32)), ("coherent", c_int32),
        ("kernel_inv_r", c_int32),
    ]


class Geometry(ctypes.Structure):
    _fields_ = [
        ("mode", c_int32), ("x0", c_double), ("y0", c_double), ("dx", c_double), ("dy", c_double),
        ("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("z", POINTER(c_double)),
        ("plane_ptr", POINTER(c_int32)), ("voxel_xy_dev", c_void_p), ("zref", c_double),
        ("alpha", POINTER(c_double)), ("xp", c_double * 3),
        ("relay_z_dev", c_void_p), ("z_mid", c_double), ("dz3", c_double), ("mz3", c_int32),
    ]


class Options(ctypes.Structure):
    _fields_ = [
        ("n_relay", c_int32), ("pad", c_double), ("sigma_os", c_double), ("tol", c_double),
        ("M", c_int32), ("freq_chunk", c_int32), ("plane_chunk", c_int32),
        ("upsample_q", c_int32), ("weights_dev", c_void_p), ("spread_tile", c_int32),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("M", c_int32), ("Mf", c_int32), ("n_freq", c_int32), ("n_relay", c_int32),
        ("kernel_width", c_int32), ("n_voxels", c_int32), ("dx", c_double), ("dy", c_double),
        ("cx", c_double), ("cy", c_double), ("beta", c_double), ("workspace_bytes", c_size_t),
        ("freq_chunk", c_int32), ("plane_chunk", c_int32), ("depth3d", c_int32),
        ("upsample_q", c_int32),
    ]


# name -> (restype, argtypes)
SIGNATURES = {
    "nursd_default_options": (None, [POINTER(Wavelet), POINTER(Geometry), POINTER(Options)]),
    "nursd_plan_create": (c_int32, [POINTER(Wavelet), POINTER(Geometry), POINTER(Options), c_void_p,
                                    c_void_p, POINTER(c_void_p)]),
    "nursd_plan_set_points": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "nursd_plan_info": (c_int32, [c_void_p, POINTER(PlanInfo)]),
    "nursd_workspace_size": (c_int32, [c_void_p, POINTER(c_size_t)]),
    "nursd_plan_destroy": (None, [c_void_p]),
    "nursd_phasor": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "nursd_spectrum": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "nursd_forward_hist": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "nursd_forward_hist_static": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "nursd_forward_phasor": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "nursd_adjoint": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                c_void_p]),
    "nursd_video_workspace_size": (c_int32, [c_void_p, POINTER(c_size_t)]),
    "nursd_forward_video": (c_int32, [c_void_p, c_void_p, c_int32, c_double, c_double, c_void_p, c_void_p, c_void_p,
                                      c_size_t, c_void_p]),
    "nursd_multi_workspace_size": (c_int32, [c_void_p, c_int32, POINTER(c_size_t)]),
    "nursd_forward_multi": (c_int32, [c_void_p, c_void_p, c_int32, POINTER(c_double), c_void_p, c_void_p, c_void_p,
                                      c_size_t, c_void_p]),
    "nursd_subsample_nearest": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p]),
    "nursd_batch_create": (c_int32, [POINTER(c_void_p), c_int32, c_int32, c_void_p, POINTER(c_void_p)]),
    "nursd_batch_workspace_size": (c_int32, [c_void_p, POINTER(c_size_t)]),
    "nursd_batch_autotune": (c_int32, [c_void_p, POINTER(c_void_p), POINTER(c_void_p), c_void_p, c_size_t,
                                       c_void_p]),
    "nursd_batch_forward": (c_int32, [c_void_p, POINTER(c_void_p), POINTER(c_void_p), c_void_p, c_size_t,
                                      c_void_p]),
    "nursd_batch_tuning": (c_int32, [c_void_p, c_char_p, c_size_t]),
    "nursd_batch_destroy": (None, [c_void_p]),
    "nursd_batch_info": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                                   POINTER(c_float), POINTER(c_size_t)]),
    "nursd_profile_begin": (c_int32, [c_void_p, ctypes.c_uint32]),
    "nursd_profile_end": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_int32)]),
    "nursd_last_error": (c_char_p, []),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libnursd.so and declare every exported entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2501_05244_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int, what: str) -> None:
    if rc != NURSD_OK:
        msg = load().nursd_last_error().decode(errors="replace")
        raise RuntimeError(f"{what} failed with {ERRORS.get(rc, rc)}: {msg}")


def c_float_p(v) -> c_void_p:
    return c_void_p(v)


__all__ = ["load", "check", "Wavelet", "Geometry", "Options", "PlanInfo", "SIGNATURES",
           "MODE_GRID", "MODE_POINTS", "MODE_SRSD", "MODE_SRSD_POINTS", "MODE_GRID3D", "c_float"]
