"""ctypes declarations of the C ABI in include/mumode.h.

Loads the in-tree ``libmumode.so``.  There is no fallback: if the library is
missing, importing this module raises, so nothing silently runs elsewhere.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmumode.so")

MM_MAXD = 6

MM_OK, MM_ERR_ARG, MM_ERR_SHAPE, MM_ERR_DTYPE, MM_ERR_ALIGN, MM_ERR_NOMEM, MM_ERR_HIP, \
    MM_ERR_UNSUPPORTED, MM_ERR_NONFINITE, MM_ERR_NODEVICE = range(10)
MM_R32, MM_R64, MM_C64, MM_C128 = range(4)
MM_PREC_FP64, MM_PREC_FP32, MM_PREC_SPLIT_BF16X3, MM_PREC_SPLIT_FP16X2, MM_PREC_BF16 = range(5)

# every symbol include/mumode.h declares
EXPORTS = [
    "mm_create", "mm_destroy", "mm_status_string", "mm_last_error", "mm_version",
    "mm_op_prepare", "mm_op_destroy", "mm_op_info",
    "mumode_apply", "mumode_expstep", "mumode_transform", "gpe_strang_step", "mm_norm2",
    "mm_profile_begin", "mm_profile_end", "ho_strang_step", "mm_energy_gpe", "mm_hermite_ho_exponential",
    "mumode_expstep_batched",
    "mm_fd2_matrix", "mm_expm", "mm_hermite_nodes", "mm_hermite_matrices",
    "mm_autotune", "mm_tune_count", "mm_tune_get", "mm_tune_clear", "mm_tune_save", "mm_tune_load",
    "mm_set_workspace", "mumode_magnus_step", "mm_expm_device",
    "mm_fd2_periodic_order", "mm_fourier_d2", "mm_pipe_flow_operators", "mm_set_option", "mm_monitor_log",
    "mm_schrodinger_fd_hamiltonian", "mm_schrodinger_fd_exponential", "mm_hermite_ho_generator",
    "gpe_strang_step_noalloc", "mm_nonuniform_neumann_d2", "mm_op_prepare_ex", "mm_op_flags",
    "mm_autotune_batched", "mm_autotune_batched_get", "vortex_strang_step",
]


class MMTensor(C.Structure):
    _fields_ = [("d", C.c_int), ("dims", C.c_int64 * MM_MAXD), ("dtype", C.c_int), ("data", C.c_void_p)]


class MMMatrix(C.Structure):
    _fields_ = [("rows", C.c_int64), ("cols", C.c_int64), ("ld", C.c_int64), ("dtype", C.c_int),
                ("data", C.c_void_p), ("on_device", C.c_int)]


def _load():
    # torch ships its own HIP runtime (soname libamdhip64.so.7).  Loading it
    # first makes the library bind to that same runtime instead of pulling in
    # a second HIP / HSA runtime from /opt/rocm, which would leave torch
    # without devices.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2103_01691_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    st = C.c_int
    P = C.c_void_p
    d = C.c_double
    sig = {
        "mm_create": (st, [C.POINTER(P), C.c_int, C.c_char_p]),
        "mm_destroy": (st, [P]),
        "mm_status_string": (C.c_char_p, [st]),
        "mm_last_error": (C.c_char_p, [P]),
        "mm_version": (C.c_char_p, []),
        "mm_op_prepare": (st, [P, C.POINTER(MMMatrix), C.c_int, C.POINTER(P)]),
        "mm_op_destroy": (st, [P, P]),
        "mm_op_prepare_ex": (st, [P, C.POINTER(MMMatrix), C.c_int, C.c_uint, C.POINTER(P)]),
        "mm_op_flags": (st, [P, C.POINTER(C.c_uint)]),
        "mm_op_info": (st, [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "mumode_apply": (st, [P, C.POINTER(MMTensor), C.POINTER(MMTensor), P, C.c_int, P]),
        "mumode_expstep": (st, [P, C.POINTER(MMTensor), C.POINTER(P), C.c_int, P]),
        "mumode_transform": (st, [P, C.POINTER(MMTensor), C.POINTER(MMTensor), C.POINTER(P), P]),
        "gpe_strang_step": (st, [P, C.POINTER(MMTensor), C.POINTER(P), d, d, C.c_int, P]),
        "gpe_strang_step_noalloc": (st, [P, C.POINTER(MMTensor), C.POINTER(P), d, d, C.c_int, P]),
        "vortex_strang_step": (st, [P, C.POINTER(MMTensor), C.POINTER(P), C.POINTER(C.POINTER(d)), d, C.c_int, P]),
        "mm_norm2": (st, [P, C.POINTER(MMTensor), d, C.POINTER(d), P]),
        "mm_profile_begin": (st, [P]),
        "ho_strang_step": (st, [P, C.POINTER(MMTensor), C.POINTER(P), C.POINTER(P), C.POINTER(C.POINTER(d)), d, d, d,
                                C.c_int, P]),
        "mumode_expstep_batched": (st, [P, C.c_int, C.POINTER(C.POINTER(MMTensor)), C.POINTER(C.POINTER(P)), C.c_int, P]),
        "mm_energy_gpe": (st, [P, C.POINTER(MMTensor), C.POINTER(P), d, d, C.POINTER(d), P]),
        "mm_hermite_ho_exponential": (st, [C.c_int, d, C.POINTER(d)]),
        "mm_profile_end": (st, [P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(d)]),
        "mm_fd2_matrix": (st, [C.c_int, d, d, C.c_int, C.POINTER(d)]),
        "mm_expm": (st, [C.c_int, C.POINTER(d), d, d, C.POINTER(d)]),
        "mm_hermite_nodes": (st, [C.c_int, C.POINTER(d), C.POINTER(d)]),
        "mm_hermite_matrices": (st, [C.c_int, C.POINTER(d), C.POINTER(d)]),
        "mm_autotune": (st, [P, C.POINTER(MMTensor), C.POINTER(P), C.c_int, P]),
        "mm_tune_count": (st, [P, C.POINTER(C.c_int)]),
        "mm_autotune_batched": (st, [P, C.c_int, C.POINTER(C.POINTER(MMTensor)), C.POINTER(C.POINTER(P)), C.c_int, P]),
        "mm_autotune_batched_get": (st, [P, C.c_int, C.c_int, C.POINTER(C.c_int)]),
        "mm_tune_get": (st, [P, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int), C.POINTER(d)]),
        "mm_tune_clear": (st, [P]),
        "mm_tune_save": (st, [P, C.c_char_p]),
        "mm_tune_load": (st, [P, C.c_char_p]),
        "mm_set_workspace": (st, [P, P, C.c_size_t]),
        "mumode_magnus_step": (st, [P, C.POINTER(MMTensor), C.POINTER(MMMatrix), C.POINTER(C.POINTER(d)),
                                    C.POINTER(d), d, C.c_int, C.c_int, P]),
        "mm_expm_device": (st, [P, C.c_int, P, d, d, P, P]),
        "mm_fd2_periodic_order": (st, [C.c_int, d, d, C.c_int, C.POINTER(d)]),
        "mm_fourier_d2": (st, [C.c_int, d, d, C.POINTER(d)]),
        "mm_set_option": (st, [P, C.c_int, C.c_int64]),
        "mm_monitor_log": (st, [P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(d)]),
        "mm_pipe_flow_operators": (st, [C.c_int, C.c_int, d, d, d, d, C.POINTER(d), C.POINTER(d)]),
        "mm_schrodinger_fd_hamiltonian": (st, [C.c_int, d, d, d, C.POINTER(d)]),
        "mm_schrodinger_fd_exponential": (st, [C.c_int, d, d, d, d, C.POINTER(d)]),
        "mm_hermite_ho_generator": (st, [C.c_int, C.POINTER(d)]),
        "mm_nonuniform_neumann_d2": (st, [C.c_int, C.POINTER(d), C.POINTER(d), C.POINTER(d)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()
