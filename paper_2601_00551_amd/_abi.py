"""ctypes mirror of include/sbp.h and loading of the in-tree libsbp.so.

Argument marshalling only: no computation of the method happens here.  The
library must have been built (``python paper_2601_00551_amd/build.py`` or
``__graft_entry__.build()``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbp.so")

SBP_OK = 0
SBP_E_ARG = -1
SBP_E_DOMAIN = -2
SBP_E_HIP = -3
SBP_E_NOMEM = -4
SBP_E_CAPACITY = -5
ERROR_NAMES = {SBP_E_ARG: "SBP_E_ARG", SBP_E_DOMAIN: "SBP_E_DOMAIN", SBP_E_HIP: "SBP_E_HIP",
               SBP_E_NOMEM: "SBP_E_NOMEM", SBP_E_CAPACITY: "SBP_E_CAPACITY"}

PROFILE_UNIFORM, PROFILE_GAUSS = 0, 1
DIR_OMNI, DIR_COS = 0, 1
SAMPLING_BIN, SAMPLING_POINT = 0, 1
X, Y, Z, P0, A = 1, 2, 4, 8, 16
XYZ, ALL, COARSE = 7, 31, 24
MAX_FRAMES = 64
MAX_TAPS = 4095

P = ctypes.c_void_p


class SbpModel(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("dt", ctypes.c_double), ("t0", ctypes.c_double),
                ("gauss_K", ctypes.c_double), ("T", ctypes.c_int32), ("f", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("directivity", ctypes.c_int32),
                ("a_softplus", ctypes.c_int32), ("sampling", ctypes.c_int32),
                ("response", ctypes.c_void_p), ("response_taps", ctypes.c_int32),
                ("response_zero", ctypes.c_int32), ("response_rows", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class SbpArray(ctypes.Structure):
    _fields_ = [("qx", P), ("qy", P), ("qz", P), ("nx", P), ("ny", P), ("nz", P),
                ("D", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class SbpBalls(ctypes.Structure):
    _fields_ = [("x", P), ("y", P), ("z", P), ("p0", P), ("a", P)]


class SbpAdamParams(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float * 5), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("step", ctypes.c_int32), ("mask", ctypes.c_uint32)]


class SbpState(ctypes.Structure):
    _fields_ = [("balls", SbpBalls), ("grad", SbpBalls), ("m", SbpBalls), ("v", SbpBalls),
                ("ball_off", P), ("F", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("B_cap", ctypes.c_int64)]


class SbpGrowthRule(ctypes.Structure):
    _fields_ = [("destroy_frac", ctypes.c_float), ("a_min", ctypes.c_float),
                ("a_split", ctypes.c_float), ("dup_frac", ctypes.c_float),
                ("dup_offset", ctypes.c_float), ("reserved", ctypes.c_int32)]


class SbpTuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("fwd_dets", "fwd_block", "fwd_bpt", "fwd_grid",
                                               "adj_dets", "adj_block", "adj_bpt", "adj_grid",
                                               "fwd_tile", "adj_tile")]


I32, I64, U32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
PM, PA, PB = ctypes.POINTER(SbpModel), ctypes.POINTER(SbpArray), ctypes.POINTER(SbpBalls)
PS, PAd, PG = ctypes.POINTER(SbpState), ctypes.POINTER(SbpAdamParams), ctypes.POINTER(SbpGrowthRule)
PT = ctypes.POINTER(SbpTuning)


class SbpGrid(ctypes.Structure):
    _fields_ = [("ox", ctypes.c_float), ("oy", ctypes.c_float), ("oz", ctypes.c_float),
                ("h", ctypes.c_float), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("reserved", ctypes.c_int32)]


PGr = ctypes.POINTER(SbpGrid)
F32 = ctypes.c_float
MLP_IN, MLP_HID, MLP_OUT, MLP_NPARAM, MLP_NWORK = 31, 256, 2, 140546, 278528

# name -> (restype, argtypes); the names are the C-ABI's entry points.
SIGNATURES = {
    "sbp_last_error": (ctypes.c_char_p, []),
    "sbp_ctx_create": (ctypes.c_int, [ctypes.POINTER(P), ctypes.c_int]),
    "sbp_ctx_destroy": (ctypes.c_int, [P]),
    "sbp_ctx_num_cus": (ctypes.c_int, [P, ctypes.POINTER(I32)]),
    "sbp_ctx_set_tuning": (ctypes.c_int, [P, PT]),
    "sbp_ctx_get_tuning": (ctypes.c_int, [P, PT]),
    "sbp_downsample": (ctypes.c_int, [P, P, I64, I32, I32, P, P]),
    "sbp_decimate": (ctypes.c_int, [P, P, I64, I32, I32, P, P]),
    "sbp_simulate_signals": (ctypes.c_int, [P, PA, PB, P, I32, I64, PM, P, I32, P]),
    "sbp_simulate_signals_noalloc": (ctypes.c_int, [P, PA, PB, P, I32, I64, PM, P, I32, P]),
    "sbp_residual_loss": (ctypes.c_int, [P, P, P, I64, I32, P, P, P]),
    "sbp_adjoint_gradients": (ctypes.c_int, [P, PA, PB, P, I32, I64, PM, P, U32, PB, P]),
    "sbp_filter_zero_grad": (ctypes.c_int, [P, PA, PB, P, I32, I64, PM, P, I32, PB, P, P,
                                            PB, PB, PB, PB, P]),
    "sbp_adam_update": (ctypes.c_int, [P, PS, PAd, P, P]),
    "sbp_step": (ctypes.c_int, [P, PA, PS, PM, P, P, PAd, P, P]),
    "sbp_step_graph_create": (ctypes.c_int, [P, PA, PS, PM, P, P, PAd, P, P, I32,
                                             ctypes.POINTER(P), P]),
    "sbp_graph_launch": (ctypes.c_int, [P, P]),
    "sbp_graph_destroy": (ctypes.c_int, [P]),
    "sbp_grow": (ctypes.c_int, [P, PS, PG, PS, ctypes.POINTER(I64), P]),
    "sbp_softplus_reparam": (ctypes.c_int, [P, PS, I32, P]),
    "sbp_response_length": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.POINTER(I32),
                                           ctypes.POINTER(I32)]),
    "sbp_response_taps": (ctypes.c_int, [P, P, P, I32, ctypes.c_double, I32, I32, P, P]),
    "sbp_response_apply": (ctypes.c_int, [P, P, I32, I32, I32, P, I64, I32, I32, I32, I32, P, P]),
    "sbp_simulate_signals_f64": (ctypes.c_int, [P, PA, PB, P, I32, I64, PM, P, I32, P]),
    "sbp_adjoint_gradients_f64": (ctypes.c_int, [P, PA, PB, P, I32, I64, PM, P, U32, PB, P]),
    # sbp_mlp.h
    "sbp_mlp_sync": (ctypes.c_int, [P, P, P, P]),
    "sbp_mlp_forward": (ctypes.c_int, [P, P, P, P, I64, P, P, P]),
    "sbp_mlp_loss": (ctypes.c_int, [P, P, P, P, I64, F32, P, P, P, P]),
    "sbp_mlp_backward": (ctypes.c_int, [P, P, P, P, P, I64, P, P, P]),
    "sbp_mlp_adam": (ctypes.c_int, [P, P, P, P, P, PAd, P, P]),
    "sbp_grid_mass": (ctypes.c_int, [P, PB, P, I64, PGr, P, P]),
    "sbp_candidates": (ctypes.c_int, [P, PGr, P, F32, F32, PB, I64, ctypes.POINTER(I64), P]),
    "sbp_features": (ctypes.c_int, [P, PGr, P, PB, I64, PB, F32, P, P]),
    "sbp_append_proposals": (ctypes.c_int, [P, PS, PB, P, I64, F32, F32, ctypes.POINTER(I64), P]),
    "sbp_merge_proposals": (ctypes.c_int, [P, PS, PB, P, P, I64, P, F32, PS, ctypes.POINTER(I64), P]),
    # sbp_image.h
    "sbp_voxelize": (ctypes.c_int, [P, PB, P, I64, PM, PGr, P, P]),
    "sbp_image_metrics": (ctypes.c_int, [P, P, P, I32, I32, I32, F32, P, P, P]),
    "sbp_mesh_inside": (ctypes.c_int, [P, P, I32, P, P, P, I64, F32, P, P, P]),
}

_LIB = None


class SbpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def lib():
    """The loaded library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2601_00551_amd/build.py "
                               "(there is no fallback path)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def check(rc):
    if rc != SBP_OK:
        raise SbpError(rc, lib().sbp_last_error().decode(errors="replace"))
    return rc
