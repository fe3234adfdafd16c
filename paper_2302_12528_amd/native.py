"""ctypes binding of liblobpcg.so (argument marshalling only).

Names mirror include/lobpcg.h.  Device buffers are torch tensors on the GPU
(passed as raw pointers); torch supplies device memory and the current stream.
The library must be built in-tree (paper_2302_12528_amd/liblobpcg.so); loading
fails loudly otherwise -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as ct
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblobpcg.so")

LOBPCG_OK = 0
LOBPCG_NOT_CONVERGED = 1
LOBPCG_ERR_INVALID_ARG = 2
LOBPCG_ERR_FACTOR_BREAKDOWN = 3
LOBPCG_ERR_ORTHO_BREAKDOWN = 4
LOBPCG_ERR_NONFINITE = 5
LOBPCG_ERR_ALLOC = 6
LOBPCG_ERR_HIP = 7
LOBPCG_ERR_STATE = 8

LOBPCG_FP64 = 0
LOBPCG_FP32 = 1
LOBPCG_FLAG_GRAPH = 1
LOBPCG_FLAG_AUTOTUNE = 2
LOBPCG_FLAG_FORCE_FP64_REDO = 4
LOBPCG_STOP_PAPER = 0
LOBPCG_STOP_NORMA = 1


class Matrix(ct.Structure):
    _fields_ = [("format", ct.c_int32), ("grid", ct.c_int32 * 3), ("n", ct.c_int64), ("nnz", ct.c_int64),
                ("rowptr", ct.c_void_p), ("colind", ct.c_void_p), ("val", ct.c_void_p),
                ("dense", ct.c_void_p), ("ld", ct.c_int64)]


ALLOC_FN = ct.CFUNCTYPE(ct.c_void_p, ct.c_size_t, ct.c_void_p)
FREE_FN = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_void_p)


class Allocator(ct.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ct.c_void_p)]


class Options(ct.Structure):
    _fields_ = [("leaf_size", ct.c_int32), ("stop_rule", ct.c_int32), ("qr_lower", ct.c_int32),
                ("flags", ct.c_int32), ("norm_a", ct.c_double), ("eig_tol", ct.c_double),
                ("subtree_levels", ct.c_int32), ("schur_wide_tiles", ct.c_int32), ("stage1_tol", ct.c_double),
                ("allocator", ct.POINTER(Allocator))]


class Info(ct.Structure):
    _fields_ = [("iters", ct.c_int32), ("n_conv", ct.c_int32), ("fallbacks", ct.c_int32), ("nlevels", ct.c_int32),
                ("norm_a", ct.c_double), ("t_symbolic", ct.c_double), ("t_factor", ct.c_double),
                ("t_solve", ct.c_double), ("nnz_factor", ct.c_double), ("factor_flops", ct.c_double),
                ("resid", ct.c_void_p), ("t_precond_gpu", ct.c_double), ("t_spmm_gpu", ct.c_double),
                ("n_precond", ct.c_int32), ("n_spmm", ct.c_int32), ("stage1_iters", ct.c_int32),
                ("stage1_exit", ct.c_int32), ("t_stage1", ct.c_double)]


# name -> (restype, argtypes); every symbol declared in include/lobpcg.h
SIGNATURES = {
    "lobpcg_setup": (ct.c_int, [ct.POINTER(Matrix), ct.c_int32, ct.c_int32, ct.c_double, ct.c_int, ct.c_void_p,
                                ct.POINTER(Options), ct.POINTER(ct.c_void_p)]),
    "lobpcg_update_values": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_void_p]),
    "lobpcg_factor": (ct.c_int, [ct.c_void_p]),
    "lobpcg_solve": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_void_p, ct.POINTER(Info)]),
    "lobpcg_setup_batched": (ct.c_int, [ct.POINTER(Matrix), ct.c_int32, ct.c_int32, ct.c_int32, ct.c_double,
                                        ct.c_int, ct.c_void_p, ct.POINTER(Options), ct.POINTER(ct.c_void_p)]),
    "lobpcg_solve_batched": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_void_p,
                                        ct.POINTER(Info)]),
    "lobpcg_batch_count": (ct.c_int32, [ct.c_void_p]),
    "lobpcg_setup_hermitian": (ct.c_int, [ct.POINTER(Matrix), ct.c_int32, ct.c_int32, ct.c_double, ct.c_int,
                                          ct.c_void_p, ct.POINTER(Options), ct.POINTER(ct.c_void_p)]),
    "lobpcg_solve_hermitian": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_void_p,
                                          ct.POINTER(Info)]),
    "lobpcg_pinvit": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_void_p, ct.POINTER(Info),
                                 ct.c_void_p]),
    "lobpcg_backward": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "lobpcg_backward_iters": (ct.c_int32, [ct.c_void_p]),
    "lobpcg_destroy": (ct.c_int, [ct.c_void_p]),
    "lobpcg_status_string": (ct.c_char_p, [ct.c_int]),
    "lobpcg_last_error": (ct.c_char_p, []),
    "lobpcg_symbolic": (ct.c_int, [ct.POINTER(Matrix), ct.c_int32, ct.c_void_p, ct.c_void_p]),
    "lobpcg_exact_fill": (ct.c_int, [ct.POINTER(Matrix), ct.c_int32, ct.c_void_p]),
    "lobpcg_get_permutation": (ct.c_int, [ct.c_void_p, ct.c_void_p]),
    "lobpcg_get_tuning": (ct.c_int, [ct.c_void_p, ct.c_void_p]),
    "lobpcg_apply_a": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_int64, ct.c_int32]),
    "lobpcg_apply_precond": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "lobpcg_mixed_qr": (ct.c_int, [ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int64, ct.c_int32, ct.c_void_p,
                                   ct.c_void_p]),
    "lobpcg_mixed_qr_noalloc": (ct.c_int, [ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int64, ct.c_int32,
                                           ct.c_void_p, ct.c_void_p]),
    "lobpcg_gram": (ct.c_int, [ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_int64, ct.c_int64, ct.c_int32, ct.c_int32,
                               ct.c_void_p, ct.c_void_p]),
    "lobpcg_syev_small": (ct.c_int, [ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
}

_lib = None


class LobpcgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def load():
    """Load the in-tree library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2302_12528_amd.build` "
                           "(there is no CPU fallback)")
    lib = ct.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    msg = load().lobpcg_last_error()
    return msg.decode() if msg else ""


def check(status: int, allow=(LOBPCG_OK,)) -> int:
    if status not in allow:
        lib = load()
        raise LobpcgError(status, f"{lib.lobpcg_status_string(status).decode()}: {last_error()}")
    return status
