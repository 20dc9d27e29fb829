"""Helpers for the GPU tests: device round trips and bitwise comparison."""
import numpy as np


def to_dev(*arrays):
    import torch

    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def to_host(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


def gpu_ksvd2(planes, plain=True, fast=False):
    import torch

    from paper_2407_13116_amd import api

    out = api.ksvd2_batch(*to_dev(*planes), plain=plain, fast=fast)
    torch.cuda.synchronize()
    return to_host(out)


def assert_bitwise(got: dict, want: dict, keys=None, idx=None, label=""):
    """Bit-for-bit equality of every output plane (NaNs must coincide)."""
    keys = keys or [k for k in want if k in got]
    for k in keys:
        a = got[k] if idx is None else got[k][idx]
        b = want[k]
        assert a.shape == b.shape, (label, k, a.shape, b.shape)
        if a.dtype.kind == "f":
            na, nb = np.isnan(a), np.isnan(b)
            assert np.array_equal(na, nb), (label, k, "NaN positions differ")
            ua = a[~na].view(np.uint64 if a.dtype == np.float64 else np.uint32)
            ub = b[~nb].view(np.uint64 if b.dtype == np.float64 else np.uint32)
            bad = np.nonzero(ua != ub)[0]
        else:
            bad = np.nonzero(a != b)[0]
        if bad.size:
            i = bad[0]
            raise AssertionError(f"{label}: plane {k}: {bad.size} mismatches, first at {i}: "
                                 f"gpu {a[i]!r} oracle {b[i]!r}")


def bit_report(got, want):
    """Count mismatching elements per plane (for diagnostics)."""
    rep = {}
    for k in want:
        if k not in got:
            continue
        a, b = got[k], want[k]
        if a.dtype.kind == "f":
            eq = (a.view(np.uint8).reshape(a.size, -1) == b.view(np.uint8).reshape(b.size, -1)).all(1)
            eq |= np.isnan(a) & np.isnan(b)
        else:
            eq = a == b
        rep[k] = int((~eq).sum())
    return rep
