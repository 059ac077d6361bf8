"""ctypes declarations of the C ABI in include/pat_nufft.h.

Loads the in-tree libpatnufft.so. There is no fallback: if the library is
missing, importing the binding raises, so nothing silently runs elsewhere.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpatnufft.so")

PAT_OK = 0
PAT_ERR_INVALID_ARGUMENT = 1
PAT_ERR_UNSUPPORTED = 2
PAT_ERR_ALLOC = 3
PAT_ERR_HIP = 4
PAT_ERR_NOT_IMPLEMENTED = 5
PAT_ERR_WORKSPACE_TOO_LARGE = 6
PAT_NOALLOC_SCRATCH_BYTES = 256 * 1024 * 1024  # the library's fixed scratch for pat_reconstruct_noalloc

PAT_FP64, PAT_FP32, PAT_FP32_KAHAN = 0, 1, 2
PAT_KERNEL_GAUSSIAN, PAT_KERNEL_KAISER_BESSEL = 0, 1
PAT_INTERP_WINDOW, PAT_INTERP_LINEAR = 0, 1
PAT_TIMING_STAGES = 6
PAT_BATCH_MAX = 64

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class PlanDesc(C.Structure):
    _fields_ = [
        ("n_sensors", C.c_int32),
        ("n_t", C.c_int32),
        ("dt", C.c_double),
        ("c", C.c_double),
        ("sensor_xy", C.POINTER(C.c_double)),
        ("sensor_h", C.POINTER(C.c_double)),
        ("nx", C.c_int32),
        ("ny", C.c_int32),
        ("nz", C.c_int32),
        ("lx", C.c_double),
        ("ly", C.c_double),
        ("lz", C.c_double),
        ("sigma_xy", C.c_double),
        ("width_xy", C.c_int32),
        ("sigma_t", C.c_double),
        ("width_t", C.c_int32),
        ("kernel", C.c_int),
        ("precision", C.c_int),
        ("temporal_interp", C.c_int),
        ("alloc", ALLOC_FN),
        ("free", FREE_FN),
        ("alloc_ctx", C.c_void_p),
    ]


class PlanInfo(C.Structure):
    _fields_ = [
        ("nx_over", C.c_int32),
        ("ny_over", C.c_int32),
        ("nt_over", C.c_int32),
        ("band_lo", C.c_int32),
        ("band_bins", C.c_int32),
        ("time_origin", C.c_int32),
        ("element_bytes", C.c_int32),
        ("spread_tiles", C.c_int32),
        ("spread_pairs", C.c_int64),
        ("workspace_bytes", C.c_size_t),
        ("table_bytes", C.c_size_t),
        ("chunk_bins", C.c_int32),
        ("rounds", C.c_int32),
        ("deconv_range_xy", C.c_double),
        ("deconv_range_t", C.c_double),
        ("forward_fused", C.c_int32),
        ("pad0", C.c_int32),
        ("spread_slots", C.c_int64),
        ("band_pairs", C.c_int64),
    ]


# every symbol the header declares, with its signature
SIGNATURES = {
    "pat_plan_desc_init": (C.c_int, [C.POINTER(PlanDesc)]),
    "nufft_plan": (C.c_int, [C.POINTER(PlanDesc), C.c_void_p, C.POINTER(C.c_void_p)]),
    "nufft_plan_workspace_size": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "pat_plan_get_info": (C.c_int, [C.c_void_p, C.POINTER(PlanInfo)]),
    "nufft_plan_destroy": (C.c_int, [C.c_void_p]),
    "pat_reconstruct": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pat_reconstruct_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pat_spectrum": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pat_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pat_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pat_forward_dxy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pat_batch_create": (C.c_int, [C.POINTER(PlanDesc), C.c_int32, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "pat_batch_groups": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "pat_batch_get_plan": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
    "pat_batch_set_grid": (C.c_int, [C.c_void_p, C.c_int32]),
    "pat_batch_reconstruct": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_void_p]),
    "pat_batch_destroy": (C.c_int, [C.c_void_p]),
    "pat_timing_begin": (C.c_int, [C.c_void_p, C.c_int32]),
    "pat_timing_begin_stages": (C.c_int, [C.c_void_p, C.c_int32, C.c_uint32]),
    "pat_timing_end": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32)]),
    "pat_status_str": (C.c_char_p, [C.c_int]),
    "pat_version": (C.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the library once and attach the signatures. Raises OSError if the
    library has not been built (run __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP runtime under the same soname: loading it
    # first makes the library bind to that one runtime. Loaded the other way
    # round, torch's tensors and the library's calls would use two runtimes
    # and the first library call on torch's memory fails.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise OSError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PatError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        msg = lib.pat_status_str(status).decode()
        super().__init__(f"{where}: {msg}")
        self.status = status


def check(status: int, where: str):
    if status != PAT_OK:
        raise PatError(status, where)
