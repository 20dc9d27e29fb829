"""ctypes loader for libksvd2.so (the HIP library; C ABI in include/ksvd2.h).

There is no fallback: if the library is missing or a tensor is not on the GPU,
the call raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libksvd2.so")

_lib = None


class KSVD2Error(RuntimeError):
    pass


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise KSVD2Error(
                f"{LIB_PATH} is not built: run `python -m paper_2407_13116_amd.build` "
                "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(LIB_PATH)
        i64, i32, p, d = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_double
        L.ksvd2_version.restype = i32
        L.ksvd2_version.argtypes = []
        L.ksvd2_last_error.restype = ctypes.c_char_p
        L.ksvd2_last_error.argtypes = []
        for name in ("ksvd2_batch_f64", "ksvd2_batch_f32", "ksvd2_batch_fast_f64",
                     "ksvd2_batch_fast_f32"):
            fn = getattr(L, name)
            fn.restype = i32
            fn.argtypes = [i64] + [p] * 15 + [p]
        L.ksvd2_svd2x2.restype = i32
        L.ksvd2_svd2x2.argtypes = [i32, i64, p, p, p, p, p, p]
        L.ksvd2_svd2x2_backward.restype = i32
        L.ksvd2_svd2x2_backward.argtypes = [i32, i64, p, p, p, p, p, p, p, d, p]
        L.ksvd2_batch_backward.restype = i32
        L.ksvd2_batch_backward.argtypes = [i32, i64] + [p] * 15 + [d, p]
        L.ksvd2c_batch.restype = i32
        L.ksvd2c_batch.argtypes = [i32, i64, p, p, p, p, p, p, p, p]
        for name in ("ksvd2_hypot_batch", "ksvd2_hypot_fast_batch"):
            fn = getattr(L, name)
            fn.restype = i32
            fn.argtypes = [i32, i64, p, p, p, p]
        if hasattr(L, "kog_sweep_batch"):
            L.kog_sweep_batch.restype = i32
            L.kog_sweep_batch.argtypes = [i32, i64, p, p, p, p, p, p, p, i32, d, i32, i32, i32, p,
                                          ctypes.c_size_t, p]
            L.kog_sweep_batch_noalloc.restype = i32
            L.kog_sweep_batch_noalloc.argtypes = [i32, i64, p, p, p, p, p, p, p, i32, d, i32, i32,
                                                  i32, p]
            L.kog_sweep_workspace_size.restype = ctypes.c_size_t
            L.kog_sweep_workspace_size.argtypes = [i32, i64, p]
            L.kog_sigma_grad.restype = i32
            L.kog_sigma_grad.argtypes = [i32, i64, p, p, p, p, p, p, p, ctypes.c_size_t, p]
            L.kog_sweep_sort.restype = i32
            L.kog_sweep_sort.argtypes = [i32, i64, p, p, p, p, p, p, ctypes.c_size_t, p]
            L.kog_rect_workspace_size.restype = ctypes.c_size_t
            L.kog_rect_workspace_size.argtypes = [i64]
            L.kog_qrcp_batch.restype = i32
            L.kog_qrcp_batch.argtypes = [i32, i64, p, p, p, p, p, p, p, p, p, ctypes.c_size_t, p]
            L.kog_qrcp_apply.restype = i32
            L.kog_qrcp_apply.argtypes = [i32, i64, p, p, p, p, p, p, p, p, p, p, p, p,
                                         ctypes.c_size_t, p]
            L.kog_sweep_tune.restype = i32
            L.kog_sweep_tune.argtypes = [i32, i32, i32]
            L.kog_sweep_set_tuning.restype = i32
            L.kog_sweep_set_tuning.argtypes = [i32, i32, i32, i32]
            L.kog_sweep_get_tuning.restype = i32
            L.kog_sweep_get_tuning.argtypes = [i32, i32, i32]
            L.kog_sweep_reset_tuning.restype = i32
            L.kog_sweep_reset_tuning.argtypes = []
        _lib = L
    return _lib


def check(rc: int, what: str = "ksvd2") -> None:
    if rc != 0:
        msg = lib().ksvd2_last_error().decode(errors="replace")
        raise KSVD2Error(f"{what} failed with status {rc}: {msg}")
