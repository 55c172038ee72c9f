"""ctypes declarations of the C ABI in include/fa.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfa.so")

FA_OK = 0
FA_WARN_NOT_CONVERGED = 1
FA_ERR_ARG = -1
FA_ERR_NO_POLY = -2
FA_ERR_BRANCH = -3
FA_ERR_HESSENBERG = -4
FA_ERR_WORKSPACE = -5
FA_ERR_HIP = -6
FA_ERR_NONFINITE = -7
FA_ERR_NO_INTERVAL = -8
FA_ERR_UNSUPPORTED = -9

FA_F64, FA_C128 = 0, 1
FA_INVSQRT, FA_SQRT = 0, 1
FA_STENCIL7, FA_WILSON4D, FA_CSR = 0, 1, 2
FA_POLY_AUTO, FA_POLY_CHEB, FA_POLY_RITZ, FA_POLY_HARMONIC, FA_POLY_LS = 0, 1, 2, 3, 4
FA_HERMITIAN, FA_FORCE_ARNOLDI, FA_PROFILE, FA_NO_FUSION, FA_MIXED = 1, 4, 8, 16, 32
FA_TWO_PASS, FA_RIGHT_PREC, FA_GRAPH, FA_CGS2, FA_FUSE2 = 64, 128, 256, 512, 1024
FA_FUSE3, FA_Q2 = 2048, 4096

EXPORTS = [
    "fa_op_device_bytes", "fa_create_csr", "fa_create_stencil", "fa_set_spectral_interval",
    "fa_get_spectral_interval", "fa_poly_workspace_bytes", "fa_poly_setup", "fa_poly_setup_ls",
    "fa_poly_get", "fa_poly_get_ls",
    "fa_workspace_bytes", "fa_apply", "fa_apply_noalloc", "fa_op_apply", "fa_poly_apply", "fa_op_info",
    "fa_destroy", "fa_status_string", "fa_dense_invsqrt_e1", "fa_dense_tridiag_invsqrt_e1",
    "fa_block_workspace_bytes", "fa_block_apply",
    "fa_server_create", "fa_server_submit", "fa_server_poll", "fa_server_wait",
    "fa_server_status", "fa_server_destroy",
]


class fa_stats(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("converged", C.c_int32), ("breakdown", C.c_int32),
        ("checks", C.c_int32), ("mvms", C.c_int64), ("mvms_setup", C.c_int64),
        ("inner_products", C.c_int64), ("est_rel_change", C.c_double), ("h_last", C.c_double),
        ("ms_total", C.c_double), ("ms_host_fH", C.c_double), ("ms_chain", C.c_double),
        ("n_chain", C.c_int64), ("chain_bytes", C.c_double), ("n_chain_terms", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class fa_block_stats(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("converged", C.c_int32), ("breakdown", C.c_int32),
        ("checks", C.c_int32), ("ns_iters", C.c_int32), ("zc", C.c_int32),
        ("graph_steps", C.c_int32), ("reserved", C.c_int32), ("mvms", C.c_int64), ("est_max", C.c_double), ("ms_total", C.c_double),
        ("ms_fH", C.c_double), ("ms_tune", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class fa_request_info(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("worker", C.c_int32), ("stats", fa_stats),
        ("t_submit_ms", C.c_double), ("t_start_ms", C.c_double), ("t_done_ms", C.c_double),
        ("ws_bytes", C.c_size_t),
    ]


class fa_server_info(C.Structure):
    _fields_ = [
        ("pending", C.c_int32), ("inflight", C.c_int32), ("peak_inflight", C.c_int32),
        ("completed", C.c_uint64), ("pool_bytes", C.c_size_t), ("bytes_inflight", C.c_size_t),
        ("peak_bytes_inflight", C.c_size_t), ("largest_free", C.c_size_t),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FAError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


_lib = None


def lib():
    """Load libfa.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2401_06684_amd.build` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, sz, i32, i64, u32, dbl = C.c_void_p, C.c_size_t, C.c_int, C.c_int64, C.c_uint32, C.c_double
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int)
    sig = {
        "fa_op_device_bytes": (sz, [i32, C.POINTER(C.c_int32), i64, i64]),
        "fa_create_csr": (i32, [C.POINTER(vp), i64, i64, vp, vp, vp, i32, u32, vp, sz, vp]),
        "fa_create_stencil": (i32, [C.POINTER(vp), i32, C.POINTER(C.c_int32), dp, i32, vp, u32,
                                    vp, sz, vp]),
        "fa_set_spectral_interval": (i32, [vp, dbl, dbl]),
        "fa_get_spectral_interval": (i32, [vp, dp, dp]),
        "fa_poly_workspace_bytes": (sz, [vp, i32, i32]),
        "fa_poly_setup": (i32, [vp, i32, i32, vp, vp, sz, vp]),
        "fa_poly_setup_ls": (i32, [vp, i32, i32, dbl, dbl, vp, vp, sz, vp]),
        "fa_poly_get": (i32, [vp, ip, ip, dp, dp, dp, dp, dp, dp]),
        "fa_poly_get_ls": (i32, [vp, C.POINTER(C.c_int64), dp, dp]),
        "fa_workspace_bytes": (sz, [vp, i32, u32]),
        "fa_apply": (i32, [vp, i32, vp, vp, i32, dbl, i32, vp, sz, u32, vp, C.POINTER(fa_stats)]),
        "fa_apply_noalloc": (i32, [vp, i32, vp, vp, i32, dbl, i32, u32, vp, C.POINTER(fa_stats)]),
        "fa_op_apply": (i32, [vp, vp, vp, vp, sz, vp]),
        "fa_poly_apply": (i32, [vp, vp, vp, vp, sz, vp]),
        "fa_op_info": (i32, [vp, C.POINTER(C.c_int64), ip]),
        "fa_destroy": (i32, [vp]),
        "fa_status_string": (C.c_char_p, [i32]),
        "fa_dense_invsqrt_e1": (i32, [i32, i32, dp, i32, dbl, dp]),
        "fa_dense_tridiag_invsqrt_e1": (i32, [i32, dp, dp, dbl, dp]),
        "fa_block_workspace_bytes": (sz, [vp, i32, i32, u32]),
        "fa_block_apply": (i32, [vp, i32, i32, vp, vp, i32, dbl, i32, vp, sz, u32, vp,
                                 C.POINTER(fa_block_stats)]),
        "fa_server_create": (i32, [C.POINTER(vp), vp, sz, i32, C.POINTER(vp)]),
        "fa_server_submit": (i32, [vp, vp, i32, vp, vp, i32, dbl, i32, u32,
                                   C.POINTER(C.c_uint64)]),
        "fa_server_poll": (i32, [vp, C.c_uint64, ip]),
        "fa_server_wait": (i32, [vp, C.c_uint64, C.POINTER(fa_request_info)]),
        "fa_server_status": (i32, [vp, C.POINTER(fa_server_info)]),
        "fa_server_destroy": (i32, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def status_string(status):
    try:
        return lib().fa_status_string(status).decode()
    except ImportError:
        return str(status)


def check(status, what):
    if status < 0:
        raise FAError(status, what)
    return status
