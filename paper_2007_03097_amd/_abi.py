"""ctypes declarations of the C ABI in include/sph.h (argument marshalling only).

Every step of the hot path runs in libsph_gfx950.so; this module only loads it and passes
pointers.  Loading fails loudly when the library has not been built -- there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph_gfx950.so")

SPH_OK, SPH_E_ARG, SPH_E_STATE, SPH_E_NOMEM, SPH_E_CAPACITY, SPH_E_DEVICE, SPH_E_NONFINITE = 0, -1, -2, -3, -4, -5, -6
SPH_FP64, SPH_FP32C = 0, 1
SPH_STEP_PRIMED, SPH_STEP_RESUME = 1, 2
SPH_ENERGY_THERMAL, SPH_ENERGY_THERMOKINETIC = 0, 1
SPH_CURVE_MORTON, SPH_CURVE_HILBERT = 0, 1
SPH_GRAVITY_QUADRUPOLE, SPH_GRAVITY_FMM = 0, 1

STATUS_NAMES = {0: "SPH_OK", -1: "SPH_E_ARG", -2: "SPH_E_STATE", -3: "SPH_E_NOMEM", -4: "SPH_E_CAPACITY",
                -5: "SPH_E_DEVICE", -6: "SPH_E_NONFINITE"}

EXPORTS = ["sph_config_default", "sph_create", "sph_destroy", "sph_workspace_size", "sph_set_workspace",
           "sph_build_tree", "sph_tree_nodes", "sph_find_neighbors", "sph_compute_density", "sph_compute_forces",
           "sph_compute_gravity", "sph_step", "sph_autotune", "sph_get_tuning", "sph_sync", "sph_last_error",
           "sph_peak_probe", "sph_timestep", "sph_key_order", "sph_step_noalloc", "sph_gravity_counts"]

SPH_NOALLOC_MAX_BYTES = 64 << 20


class sph_config(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("gamma", ctypes.c_double), ("av_alpha", ctypes.c_double),
                ("av_beta", ctypes.c_double), ("av_eps", ctypes.c_double), ("h_coeff", ctypes.c_double),
                ("adaptive_h", ctypes.c_int32), ("G", ctypes.c_double), ("soft_eps", ctypes.c_double),
                ("theta", ctypes.c_double), ("leaf_size", ctypes.c_int32), ("group_size", ctypes.c_int32),
                ("nbr_capacity", ctypes.c_int32), ("stream", ctypes.c_void_p), ("energy_form", ctypes.c_int32),
                ("key_curve", ctypes.c_int32), ("gravity_scheme", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32)]


_dp = ctypes.c_void_p  # device pointers are passed as integers


class sph_particles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_seg", ctypes.c_int32), ("seg_offsets", ctypes.POINTER(ctypes.c_int64)),
                ("x", _dp), ("y", _dp), ("z", _dp), ("vx", _dp), ("vy", _dp), ("vz", _dp), ("m", _dp), ("h", _dp),
                ("u", _dp), ("ax", _dp), ("ay", _dp), ("az", _dp), ("dudt", _dp),
                ("seg_dt", ctypes.POINTER(ctypes.c_double))]


class SPHError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load the HIP library (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2007_03097_amd/build.py "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    import torch  # noqa: F401  (loads the HIP runtime the library links against)
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    ctx_p = ctypes.c_void_p
    i32, i64, u32, dbl, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double, ctypes.c_size_t
    L.sph_config_default.argtypes = [P(sph_config)]
    L.sph_config_default.restype = None
    L.sph_create.argtypes = [P(sph_config), i64, i32, P(ctx_p)]
    L.sph_destroy.argtypes = [ctx_p]
    L.sph_workspace_size.argtypes = [ctx_p, P(sz)]
    L.sph_set_workspace.argtypes = [ctx_p, ctypes.c_void_p, sz]
    L.sph_build_tree.argtypes = [ctx_p, P(sph_particles), P(dbl), _dp, _dp]
    L.sph_tree_nodes.argtypes = [ctx_p, i64, _dp, _dp, _dp, _dp, _dp, P(i64)]
    L.sph_find_neighbors.argtypes = [ctx_p, _dp, _dp, i64, P(i64)]
    L.sph_compute_density.argtypes = [ctx_p, _dp, _dp, _dp, _dp]
    L.sph_compute_forces.argtypes = [ctx_p, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.sph_compute_gravity.argtypes = [ctx_p, _dp, _dp, _dp, _dp]
    L.sph_step.argtypes = [ctx_p, P(sph_particles), dbl, i32, u32, P(dbl)]
    L.sph_step_noalloc.argtypes = [ctx_p, P(sph_particles), dbl, i32, u32, P(dbl)]
    L.sph_autotune.argtypes = [ctx_p, P(sph_particles), dbl, ctypes.c_char_p]
    L.sph_get_tuning.argtypes = [ctx_p, P(i32), P(i32), P(i32)]
    L.sph_sync.argtypes = [ctx_p]
    L.sph_last_error.argtypes = [ctx_p]
    L.sph_last_error.restype = ctypes.c_char_p
    L.sph_peak_probe.argtypes = [i32, _dp, i64, i32, ctypes.c_void_p]
    L.sph_timestep.argtypes = [ctx_p, P(dbl)]
    L.sph_key_order.argtypes = [ctx_p, _dp, _dp]
    L.sph_gravity_counts.argtypes = [ctx_p, P(i64), P(i64)]
    for name in EXPORTS:
        if name not in ("sph_config_default", "sph_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L
