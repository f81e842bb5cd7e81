"""ctypes binding of libgfft.so: the C ABI of include/gfft.h, same names.

Argument marshalling only.  Every transform step runs in the HIP kernels of
libgfft.so; there is no fallback: if the library is missing it is built (or
an error is raised), never replaced.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# GFFT_LIB names another build of the same sources (the host-sanitized build
# of the CPU tests); by default the in-tree libgfft.so
LIB_PATH = os.environ.get("GFFT_LIB") or os.path.join(HERE, "libgfft.so")

GFFT_OK = 0
GFFT_E_INVALID_ARG = -1
GFFT_E_UNSUPPORTED = -2
GFFT_E_ALIGN = -3
GFFT_E_NOMEM = -4
GFFT_E_HIP = -5
GFFT_E_NO_DEVICE = -6

GFFT_F64 = 0
GFFT_F32 = 1

GFFT_FUSE_PACK = 1 << 0
GFFT_MFMA_BF16X2 = 1 << 1
GFFT_MFMA_BF16X3 = 1 << 2
GFFT_INPLACE = 1 << 3
GFFT_PACK_PAPER_ORDER = 1 << 4

# Every symbol include/gfft.h declares.
EXPORTS = (
    "gfft_plan_create", "gfft_pencil_plan_create", "gfft_plan_destroy", "gfft_plan_query",
    "gfft_exec_r2c", "gfft_exec_c2r", "gfft_exec_r2c_adjoint",
    "gfft_exec_c2r_adjoint", "gfft_pack_slab_for_alltoall",
    "gfft_unpack_slab_from_alltoall", "gfft_exec_x_c2c",
    "gfft_exec_z_r2c", "gfft_exec_y_c2c", "gfft_exec_z_c2r",
    "gfft_device_copy", "gfft_exec_pass_copy", "gfft_status_string", "gfft_version",
)


class gfft_plan_sizes(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "n", "slab_x", "ranks", "batch", "k", "real_bytes", "complex_bytes",
        "pencil_bytes", "chunk_bytes", "grid_r", "grid_c", "col", "y_local", "kz_width")]


class GfftError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} (status {status})")


_lib = None


def load(path: str = LIB_PATH):
    """Load libgfft.so (building it in-tree first if it is absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        from . import build
        build.build()
    lib = ctypes.CDLL(path)
    vp, i64, i32, u32, dbl = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                              ctypes.c_uint32, ctypes.c_double)
    sig = {
        "gfft_plan_create": [ctypes.POINTER(vp), i64, i32, i64, i64, u32],
        "gfft_pencil_plan_create": [ctypes.POINTER(vp), i64, i32, i64, i64, i64, i64, u32],
        "gfft_plan_destroy": [vp],
        "gfft_plan_query": [vp, ctypes.POINTER(gfft_plan_sizes)],
        "gfft_exec_r2c": [vp, vp, vp, vp],
        "gfft_exec_c2r": [vp, vp, vp, dbl, vp],
        "gfft_exec_r2c_adjoint": [vp, vp, vp, dbl, vp],
        "gfft_exec_c2r_adjoint": [vp, vp, vp, dbl, vp],
        "gfft_pack_slab_for_alltoall": [vp, vp, vp, vp],
        "gfft_unpack_slab_from_alltoall": [vp, vp, vp, vp],
        "gfft_exec_x_c2c": [vp, vp, i32, vp],
        "gfft_exec_z_r2c": [vp, vp, vp, dbl, i32, vp],
        "gfft_exec_y_c2c": [vp, vp, i32, vp],
        "gfft_exec_z_c2r": [vp, vp, vp, dbl, i32, vp],
        "gfft_device_copy": [vp, vp, i64, vp],
        "gfft_exec_pass_copy": [vp, i32, vp, vp],
        "gfft_status_string": [i32],
        "gfft_version": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = i32
    lib.gfft_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().gfft_status_string(int(status)).decode()


def check(status: int, where: str) -> None:
    if status != GFFT_OK:
        raise GfftError(status, where)


# Thin same-name wrappers over raw handles and integer addresses.

def gfft_plan_create(n, dtype, slab_x, batch, flags):
    h = ctypes.c_void_p()
    st = load().gfft_plan_create(ctypes.byref(h), n, dtype, slab_x, batch, flags)
    return st, h


def gfft_pencil_plan_create(n, dtype, grid_r, grid_c, col, batch, flags):
    h = ctypes.c_void_p()
    st = load().gfft_pencil_plan_create(ctypes.byref(h), n, dtype, grid_r, grid_c, col, batch,
                                        flags)
    return st, h


def gfft_plan_destroy(plan):
    return load().gfft_plan_destroy(plan)


def gfft_plan_query(plan):
    s = gfft_plan_sizes()
    st = load().gfft_plan_query(plan, ctypes.byref(s))
    return st, s


def gfft_exec_r2c(plan, in_real, out_cplx, stream):
    return load().gfft_exec_r2c(plan, in_real, out_cplx, stream)


def gfft_exec_c2r(plan, in_cplx, out_real, scale, stream):
    return load().gfft_exec_c2r(plan, in_cplx, out_real, scale, stream)


def gfft_exec_r2c_adjoint(plan, in_cplx, out_real, scale, stream):
    return load().gfft_exec_r2c_adjoint(plan, in_cplx, out_real, scale, stream)


def gfft_exec_c2r_adjoint(plan, in_real, out_cplx, scale, stream):
    return load().gfft_exec_c2r_adjoint(plan, in_real, out_cplx, scale, stream)


def gfft_pack_slab_for_alltoall(plan, slab, send, stream):
    return load().gfft_pack_slab_for_alltoall(plan, slab, send, stream)


def gfft_unpack_slab_from_alltoall(plan, recv, slab, stream):
    return load().gfft_unpack_slab_from_alltoall(plan, recv, slab, stream)


def gfft_exec_x_c2c(plan, pencil, sign, stream):
    return load().gfft_exec_x_c2c(plan, pencil, sign, stream)


def gfft_exec_z_r2c(plan, in_real, out_cplx, scale, weighted, stream):
    return load().gfft_exec_z_r2c(plan, in_real, out_cplx, scale, weighted, stream)


def gfft_exec_y_c2c(plan, data, sign, stream):
    return load().gfft_exec_y_c2c(plan, data, sign, stream)


def gfft_exec_z_c2r(plan, in_cplx, out_real, scale, weighted, stream):
    return load().gfft_exec_z_c2r(plan, in_cplx, out_real, scale, weighted, stream)


def gfft_device_copy(dst, src, nbytes, stream):
    return load().gfft_device_copy(dst, src, nbytes, stream)


def gfft_exec_pass_copy(plan, axis, data, stream):
    return load().gfft_exec_pass_copy(plan, axis, data, stream)


def gfft_status_string(status):
    return status_string(status)


def gfft_version():
    return load().gfft_version()
