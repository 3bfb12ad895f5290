"""ctypes declarations of the C ABI in ``include/dec_bpm.h`` (argument marshalling only).

torch is imported before the library is loaded so that the library binds to
the HIP runtime torch already holds (one runtime per process).
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede loading the library)

from .build_ext import LIB

c_int, c_i32, c_i64, c_dbl, c_vp, c_sz = (ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                          ctypes.c_void_p, ctypes.c_size_t)
P = ctypes.POINTER

OK, EINVAL, EMESH, EUNSTABLE, ENOMEM, EHIP, ENONFINITE, EWORKSPACE, ENODEVICE = 0, -1, -2, -3, -4, -5, -6, -7, -8
C64, C128 = 1, 2
NL_DEC, NL_LUMPED = 0, 1
OP_L, OP_L2, OP_H = 0, 1, 2
K_KERR, K_STAGE, K_LAP, K_TILE_A, K_TILE_B, K_STEP, K_PERSIST, K_UNSPLIT, K_DP5, K_MODE, K_DP5_PERSIST, \
    K_MODE_PERSIST, K_UNSPLIT_PERSIST, NUM_KERNELS = range(14)

ERROR_NAMES = {EINVAL: "EINVAL", EMESH: "EMESH", EUNSTABLE: "EUNSTABLE", ENOMEM: "ENOMEM", EHIP: "EHIP",
               ENONFINITE: "ENONFINITE", EWORKSPACE: "EWORKSPACE", ENODEVICE: "ENODEVICE"}


class Options(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("dtype", c_i32),
        ("p1", c_dbl),
        ("beta4", c_dbl),
        ("nonlinearity", c_i32),
        ("reorder", c_i32),
        ("chi_tri", P(c_dbl)),
        ("host_only", c_i32),
        ("block_size", c_i32),
        ("steps_per_graph", c_i32),
        ("pml_r0", c_dbl),
        ("pml_r1", c_dbl),
        ("pml_sigma", c_dbl),
        ("p3", c_dbl),
        ("p4", c_dbl),
        ("nl_kind", c_i32),
        ("nl_param", c_dbl),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [("block_size", c_i32), ("steps_per_graph", c_i32), ("fused", c_i32), ("tile_block", c_i32),
                ("xcd_remap", c_i32)]


class DecBpmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


# (name, restype, argtypes)
_SIGNATURES = [
    ("dec_bpm_default_options", None, [P(Options)]),
    ("dec_bpm_last_error", ctypes.c_char_p, []),
    ("dec_bpm_version", ctypes.c_char_p, []),
    ("dec_bpm_create", c_int, [P(c_dbl), c_i64, P(c_i32), c_i64, P(c_dbl), P(c_dbl), P(Options), P(c_vp)]),
    ("dec_bpm_destroy", None, [c_vp]),
    ("dec_bpm_sizes", c_int, [c_vp, P(c_i64), P(c_i64), P(c_i64), P(c_i64)]),
    ("dec_bpm_spectral_radius", c_int, [c_vp, P(c_dbl)]),
    ("dec_bpm_export_operators", c_int, [c_vp, P(c_dbl), P(c_dbl), P(c_dbl), P(c_i64), P(c_i64), P(c_i32),
                                         P(c_dbl), P(c_dbl)]),
    ("dec_bpm_set_index_perturbation", c_int, [c_vp, c_vp, c_vp]),
    ("dec_bpm_apply", c_int, [c_vp, c_int, c_vp, c_vp, c_vp]),
    ("dec_bpm_kerr_step", c_int, [c_vp, c_vp, c_dbl, c_dbl, c_vp]),
    ("dec_bpm_linear_step", c_int, [c_vp, c_vp, c_dbl, c_vp]),
    ("dec_bpm_propagate", c_int, [c_vp, c_vp, c_dbl, c_i64, c_dbl, c_vp]),
    ("dec_bpm_propagate_noalloc", c_int, [c_vp, c_vp, c_dbl, c_i64, c_dbl, c_vp]),
    ("dec_bpm_propagate_unsplit", c_int, [c_vp, c_vp, c_dbl, c_i64, c_dbl, c_vp]),
    ("dec_bpm_export_pml", c_int, [c_vp, P(c_dbl), P(c_dbl)]),
    ("dec_bpm_vertex_tiles", c_int, [c_vp, P(c_i32), P(c_i32)]),
    ("dec_bpm_find_mode", c_int, [c_vp, c_vp, c_dbl, c_dbl, c_dbl, c_dbl, c_i64, ctypes.POINTER(c_dbl),
                                  ctypes.POINTER(c_dbl), ctypes.POINTER(c_i64), c_vp]),
    ("dec_bpm_propagate_adaptive", c_int, [c_vp, c_vp, c_dbl, c_dbl, c_dbl, c_dbl, c_dbl, c_i64,
                                           ctypes.POINTER(c_i64), ctypes.POINTER(c_i64),
                                           ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl), c_vp]),
    ("dec_bpm_check_finite", c_int, [c_vp, c_vp]),
    ("dec_bpm_diagnostics", c_int, [c_vp, c_vp, c_dbl, P(c_dbl), P(c_dbl), c_vp]),
    ("dec_bpm_overlap", c_int, [c_vp, c_vp, c_vp, P(c_dbl), P(c_dbl), c_vp]),
    ("dec_bpm_workspace_size", c_int, [c_vp, c_i64, c_i64, P(c_sz)]),
    ("dec_bpm_forward_checkpointed", c_int, [c_vp, c_vp, c_dbl, c_i64, c_dbl, c_i64, c_vp, c_sz, c_vp]),
    ("dec_bpm_adjoint", c_int, [c_vp, c_vp, c_dbl, c_i64, c_dbl, c_i64, c_vp, c_sz, c_vp, c_vp, c_vp]),
    ("dec_bpm_batch_check_finite", c_int, [c_vp, c_vp]),
    ("dec_bpm_batch_create", c_int, [P(c_vp), c_i32, P(c_i32), P(c_vp)]),
    ("dec_bpm_batch_destroy", None, [c_vp]),
    ("dec_bpm_batch_size", c_int, [c_vp, P(c_i64)]),
    ("dec_bpm_batch_propagate", c_int, [c_vp, c_vp, c_dbl, c_i64, c_dbl, c_vp]),
    ("dec_bpm_autotune", c_int, [c_vp, c_dbl, c_dbl, c_vp]),
    ("dec_bpm_batch_autotune", c_int, [c_vp, c_dbl, c_dbl, c_vp]),
    ("dec_bpm_get_tuning", c_int, [c_vp, P(Tuning)]),
    ("dec_bpm_set_tuning", c_int, [c_vp, P(Tuning)]),
    ("dec_bpm_batch_get_tuning", c_int, [c_vp, P(Tuning)]),
    ("dec_bpm_batch_set_tuning", c_int, [c_vp, P(Tuning)]),
    ("dec_bpm_time_kernels", c_int, [c_vp, c_dbl, c_dbl, c_i32, P(c_dbl), P(c_dbl), c_vp]),
    ("dec_bpm_batch_time_kernels", c_int, [c_vp, c_dbl, c_dbl, c_i32, P(c_dbl), P(c_dbl), c_vp]),
]

SYMBOLS = [s[0] for s in _SIGNATURES]

_lib = None


def lib():
    """Load the native library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"native library {LIB} is missing: build it with __graft_entry__.build() "
                               "or python -m paper_2608_03587_amd.build_ext")
        handle = ctypes.CDLL(LIB)
        for name, res, args in _SIGNATURES:
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(rc: int) -> None:
    if rc != OK:
        raise DecBpmError(rc, lib().dec_bpm_last_error().decode(errors="replace"))
