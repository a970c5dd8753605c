"""ctypes declarations of the C ABI in include/hgl.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhgl.so")

HGL_OK = 0
HGL_NOT_CONVERGED = 1
HGL_EINVAL = -1
HGL_ENOMEM = -2
HGL_EDEVICE = -3
HGL_EBREAKDOWN = -4
HGL_ECHOLQR = -5
HGL_EUNSUPPORTED = -6

HGL_F64 = 0
HGL_F32 = 1
HGL_CG_PLAIN_F64 = 0
HGL_CG_F32_F64DOT_RR = 1

_STATUS_NAMES = {0: "HGL_OK", 1: "HGL_NOT_CONVERGED", -1: "HGL_EINVAL", -2: "HGL_ENOMEM",
                 -3: "HGL_EDEVICE", -4: "HGL_EBREAKDOWN", -5: "HGL_ECHOLQR", -6: "HGL_EUNSUPPORTED"}


class CgOpts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("x0_given", C.c_int32), ("rr_period", C.c_int32), ("chunk", C.c_int32),
                ("graph", C.c_int32), ("tune", C.c_int32)]


class RsvdOpts(C.Structure):
    _fields_ = [("k", C.c_int32), ("p", C.c_int32), ("q", C.c_int32), ("sketch", C.c_int32),
                ("seed", C.c_uint64), ("refine_tol", C.c_double), ("max_refine", C.c_int32),
                ("chunk", C.c_int32), ("scheme", C.c_int32)]


# hgl_allocator: device memory of a handle from the caller (torch's caching allocator)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


HGL_SKETCH_BF16 = 0
HGL_SKETCH_F64 = 1
HGL_RSVD_SUBSPACE = 0
HGL_RSVD_POWER = 1


P = C.c_void_p
I32 = C.c_int32
I64 = C.c_int64
D = C.c_double
I32P = C.POINTER(C.c_int32)
DP = C.POINTER(C.c_double)
I64P = C.POINTER(C.c_int64)

# name -> (restype, argtypes); every entry point the header declares
SIGNATURES = {
    "hgl_version": (C.c_int, []),
    "hgl_last_error": (C.c_char_p, []),
    "hgl_build_laplacian": (C.c_int, [I32, I32, I64, P, P, P, C.POINTER(Allocator), C.POINTER(P), P]),
    "hgl_build_laplacian_batched": (C.c_int, [I32, I32P, I32P, I64, P, P, P, C.POINTER(Allocator), C.POINTER(P),
                                              P]),
    "hgl_set_weights": (C.c_int, [P, P, P]),
    "hgl_destroy": (None, [P]),
    "hgl_get_sizes": (C.c_int, [P, I32P, I32P, C.POINTER(C.c_int64), I32P]),
    "hgl_get_partition": (C.c_int, [P, I32P, I32P, I32P, I32P]),
    "hgl_get_gather_shape": (C.c_int, [P, I32P]),
    "hgl_get_cg_stats": (C.c_int, [P, I32P]),
    "hgl_get_operator": (C.c_int, [P, P, P, P, P, P, P]),
    "hgl_apply": (C.c_int, [P, D, I32, P, I64, P, I64, I32, P]),
    "hgl_apply_noalloc": (C.c_int, [P, D, I32, P, I64, P, I64, I32, P]),
    "hgl_cg_solve": (C.c_int, [P, D, C.POINTER(CgOpts), P, I64, P, I64, I32, I32P, DP, P]),
    "hgl_cg_solve_batched": (C.c_int, [P, DP, C.POINTER(CgOpts), P, I64, P, I64, I32, I32P, DP, P]),
    "hgl_cg_solve_wg": (C.c_int, [P, D, C.POINTER(CgOpts), P, I64, P, I64, I32, I32P, DP, P]),
    "hgl_cg_solve_wg_batched": (C.c_int, [P, DP, C.POINTER(CgOpts), P, I64, P, I64, I32, I32P, DP, P]),
    "hgl_peak_copy": (C.c_int, [P, P, I64, P]),
    "hgl_peak_mfma_bf16": (C.c_int, [P, I32, I32, P]),
    "hgl_block_rsvd": (C.c_int, [P, I32, I32P, C.POINTER(RsvdOpts), P, P, P, P]),
    "hgl_block_rsvd_invert": (C.c_int, [P, D, I32, I32P, C.POINTER(RsvdOpts), P, P, I64, P, I64, I32, P,
                                        I32P, DP, P]),
    "hgl_sketch_gaussian": (C.c_int, [I64, I32, C.c_uint64, P, P]),
    "hgl_philox4x32_10": (C.c_int, [I64, P, C.c_uint64, P, P]),
    "hgl_block_schur_inverse": (C.c_int, [P, D, I32, I32P, I32, P, DP, P]),
    "hgl_block_schur_invert": (C.c_int, [P, D, I32, I32P, I32, D, I32, I32, P, I64, P, I64, I32, I32P, DP, P]),
    "hgl_block_schur_plan": (C.c_int, [I32, I32P, I32, I64P, I64P, I64P, I32P, I64P, I64P]),
    "hgl_weight_grad": (C.c_int, [P, D, D, P, I64, P, I64, P, I64, I32, C.POINTER(CgOpts), P, P, I64, I32P, DP, P]),
    "hgl_project_simplex": (C.c_int, [P, P, I32, P]),
    "hgl_projected_gradient_step": (C.c_int, [P, P, D, I32, P, P, P]),
    "hgl_active_set_step": (C.c_int, [P, P, D, I32, P, P, P, DP, P]),
    "hgl_profile": (C.c_int, [P, I32]),
    "hgl_profile_read": (C.c_int, [P, I32, C.POINTER(C.c_int64), DP]),
}

_lib = None


class HglError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        self.status = status
        super().__init__(f"{func} -> {_STATUS_NAMES.get(status, status)}: {msg}")


def load(path: str = LIB_PATH):
    """Load libhgl.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} is not built; run "
                          "`python -m paper_1908_08281_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        if not hasattr(lib, name):
            continue
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status: int, func: str) -> int:
    if status < 0:
        msg = _lib.hgl_last_error().decode(errors="replace") if _lib else ""
        raise HglError(status, func, msg)
    return status
