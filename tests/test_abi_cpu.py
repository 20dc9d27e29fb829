"""The C ABI library (CPU-side checks, no GPU needed).

* libksvd2.so loads and exports every function that include/*.h declares;
* invalid arguments are rejected before anything is enqueued (status codes and the
  last-error message), which needs no device.
"""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", txt, re.M):
            name = m.group(1)
            if name not in ("if", "while", "for", "return", "sizeof"):
                names.add(name)
    return names


@pytest.fixture(scope="module")
def L():
    from paper_2407_13116_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_2407_13116_amd import build

        build.build()
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = _declared_functions()
    assert {"ksvd2_batch_f64", "ksvd2_batch_f32", "ksvd2_batch_backward", "ksvd2_svd2x2"} <= names
    for n in sorted(names):
        assert hasattr(L, n), f"{n} declared in include/ but not exported"
    assert L.ksvd2_version() >= 1


def test_invalid_arguments_rejected(L):
    p = ctypes.c_void_p(64)  # aligned, never dereferenced: validation fails first
    rc = L.ksvd2_batch_f64(-1, *([p] * 13), None, None, None)
    assert rc == -1 and b"batch" in L.ksvd2_last_error()
    rc = L.ksvd2_batch_f64(4, None, *([p] * 12), None, None, None)
    assert rc == -1 and b"g11" in L.ksvd2_last_error()
    rc = L.ksvd2_batch_f64(4, ctypes.c_void_p(65), *([p] * 12), None, None, None)
    assert rc == -1 and b"aligned" in L.ksvd2_last_error()
    assert L.ksvd2_batch_f64(0, *([None] * 15), None) == 0          # empty batch: no-op
    assert L.ksvd2_svd2x2(7, 4, p, p, p, p, None, None) == -2
    assert L.ksvd2_svd2x2_backward(1, 4, p, p, p, None, None, None, p, -1.0, None) == -1
    assert L.ksvd2_svd2x2_backward(5, 4, p, p, p, None, None, None, p, 0.0, None) == -2
    planes = [p] * 7 + [None] * 4 + [p] * 4          # cu..s2, ds1 ds2 dU dV, dg planes
    assert L.ksvd2_batch_backward(1, 4, *planes, -1.0, None) == -1
    assert b"tau" in L.ksvd2_last_error()
    assert L.ksvd2_batch_backward(5, 4, *planes, 0.0, None) == -2
    bad = list(planes)
    bad[4] = None                                   # info is required (determinant signs)
    assert L.ksvd2_batch_backward(1, 4, *bad, 0.0, None) == -1
    assert b"info" in L.ksvd2_last_error()
    assert L.ksvd2_batch_backward(1, 0, *([None] * 15), 0.0, None) == 0
    assert L.ksvd2_hypot_batch(1, -3, p, p, p, None) == -1


def test_binding_refuses_cpu_tensors():
    import torch

    from paper_2407_13116_amd import KSVD2Error, api

    x = torch.zeros(4, dtype=torch.float64)
    with pytest.raises(KSVD2Error):
        api.ksvd2_batch(x, x, x, x)


def test_sweep_arguments_rejected(L):
    import numpy as np

    n = np.array([4, 5], dtype=np.int32)          # odd order
    off = np.array([0, 16], dtype=np.int64)
    p = ctypes.c_void_p(256)
    args = lambda nn, mode, ws_bytes, ordering=0: (1, 2, nn.ctypes.data_as(ctypes.c_void_p),
                                                   off.ctypes.data_as(ctypes.c_void_p), p, p, p,
                                                   None, None, 3, 1.0, 0, mode, ordering, p,
                                                   ws_bytes, None)
    assert L.kog_sweep_batch(*args(n, 1, 1 << 20)) == -1
    assert b"even" in L.ksvd2_last_error()
    n2 = np.array([4, 6], dtype=np.int32)
    assert L.kog_sweep_batch(*args(n2, 0, 16)) == -4                 # workspace too small
    need = L.kog_sweep_workspace_size(1, 2, n2.ctypes.data_as(ctypes.c_void_p))
    assert need >= 8 * (4 * 4 + 6 * 6)                                # holds a second G
    assert L.kog_sweep_batch(*args(n2, 2, need)) == -1                # graph mode, null stream
    assert L.kog_sweep_batch(*args(n2, 7, need)) == -1                # bad mode
    assert L.kog_sweep_batch(*args(n2, 1, need, 3)) == -1             # bad ordering
    assert b"ordering" in L.ksvd2_last_error()
    assert L.kog_sweep_tune(1, 9, 256) == -1 and L.kog_sweep_tune(1, 0, 300) == -1


def test_sweep_tuning_table(L):
    """The tuning knobs: defaults, per-bucket and all-bucket settings, range checks."""
    try:
        assert L.kog_sweep_reset_tuning() == 0
        assert [L.kog_sweep_get_tuning(1, b, 0) for b in range(5)] == [256, 512, 512, 512, 1024]
        assert [L.kog_sweep_get_tuning(0, b, 0) for b in range(5)] == [256, 512, 512, 1024, 1024]
        assert L.kog_sweep_get_tuning(0, 2, 1) == 128                  # chunk
        assert L.kog_sweep_get_tuning(0, 2, 2) == 1 and L.kog_sweep_get_tuning(0, 2, 3) == 1
        assert L.kog_sweep_get_tuning(0, 2, 4) == 0                    # rows: as many as fit
        assert L.kog_sweep_set_tuning(1, -1, 1, 32) == 0
        assert [L.kog_sweep_get_tuning(1, b, 1) for b in range(5)] == [32] * 5
        assert L.kog_sweep_get_tuning(0, 0, 1) == 128                  # the other dtype
        assert L.kog_sweep_set_tuning(1, 3, 4, 24) == 0 and L.kog_sweep_get_tuning(1, 3, 4) == 24
        assert L.kog_sweep_set_tuning(1, 0, 1, 48) == -1               # not a power of two
        assert L.kog_sweep_set_tuning(1, 0, 1, 256) == -1              # above 128
        assert L.kog_sweep_set_tuning(1, 0, 2, 2) == -1
        assert L.kog_sweep_set_tuning(1, 0, 9, 0) == -1
        assert L.kog_sweep_set_tuning(1, 5, 0, 256) == -1
        assert L.kog_sweep_set_tuning(3, 0, 0, 256) == -2
        assert L.kog_sweep_get_tuning(1, 0, 7) < 0
        assert L.kog_sweep_tune(1, 2, 1024) == 0 and L.kog_sweep_get_tuning(1, 2, 0) == 1024
        assert L.kog_sweep_tune(1, -1, 256) == -1
    finally:
        L.kog_sweep_reset_tuning()


def test_autotuner_starts_from_the_library_defaults(L):
    """The autotuner's starting point per dtype and order bucket is the library's own
    default schedule (its search and its 'ms_default' figure assume so)."""
    import torch

    from paper_2407_13116_amd import autotune

    knobs = {"block": 0, "chunk": 1, "two": 2, "inplace": 3, "rows": 4}
    try:
        assert L.kog_sweep_reset_tuning() == 0
        for dt, tdt in ((1, torch.float64), (0, torch.float32)):
            for b in range(5):
                want = autotune._default(b, tdt)
                got = {k: L.kog_sweep_get_tuning(dt, b, v) for k, v in knobs.items()}
                assert got == want, (dt, b, got, want)
    finally:
        L.kog_sweep_reset_tuning()

def test_sigma_grad_arguments_rejected(L):
    """kog_sigma_grad: argument errors before any device work (no GPU needed), and the
    workspace size function covers its descriptor and workgroup schedule."""
    import numpy as np

    n = np.array([4, 0], dtype=np.int32)
    off = np.array([0, 16], dtype=np.int64)
    p = ctypes.c_void_p(256)
    args = lambda nn, ws_bytes, dtype=1, nmat=2: (dtype, nmat, nn.ctypes.data_as(ctypes.c_void_p),
                                                  off.ctypes.data_as(ctypes.c_void_p), p, p, p, p,
                                                  p, ws_bytes, None)
    assert L.kog_sigma_grad(*args(n, 1 << 20)) == -1                  # order 0
    assert b"order" in L.ksvd2_last_error()
    assert L.kog_sigma_grad(*args(n, 1 << 20, nmat=-1)) == -1
    assert L.kog_sigma_grad(*args(n, 1 << 20, nmat=0)) == 0           # empty: no-op
    assert L.kog_sigma_grad(*args(n, 1 << 20, dtype=3)) == -2
    n2 = np.array([4, 300], dtype=np.int32)
    assert L.kog_sigma_grad(*args(n2, 64)) == -4                      # workspace too small
    need = L.kog_sweep_workspace_size(1, 2, n2.ctypes.data_as(ctypes.c_void_p))
    # descriptor (n, off, soff) and the schedule: at most 8 lists of all 1 + 9 tiles
    assert need >= 256 * 3 + 8 * 8 * 10
