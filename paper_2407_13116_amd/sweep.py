"""Batched two-sided Kogbetliantz sweep over many square matrices (C ABI
kog_sweep_batch / kog_sigma_grad in include/ksvd2.h).

Marshalling only: packing a list of matrices into one column-major device
buffer, the workspace, and the stream (the hipGraph mode needs a non-null
stream, so it runs on a side stream ordered after the caller's).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib

_DT = {torch.float32: 0, torch.float64: 1}
MODES = {"plain": 0, "persistent": 1, "graph": 2}
ORDERINGS = {"round-robin": 0, "modulus": 1, "dynamic": 2}


class Packed:
    """Square matrices packed column-major into one flat device tensor."""

    def __init__(self, mats, dtype=None, device="cuda"):
        mats = [np.asarray(m) for m in mats]
        dtype = dtype or mats[0].dtype
        self.n = np.array([m.shape[0] for m in mats], dtype=np.int32)
        sizes = self.n.astype(np.int64) ** 2
        self.off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        self.soff = np.concatenate([[0], np.cumsum(self.n.astype(np.int64))[:-1]]).astype(np.int64)
        flat = np.concatenate([np.asarray(m, dtype=dtype).ravel(order="F") for m in mats])
        self.G = torch.from_numpy(flat).to(device)
        self.dtype = self.G.dtype

    def unpack(self, flat):
        """Device flat tensor (G, U or V layout) -> list of numpy matrices."""
        h = flat.detach().cpu().numpy()
        return [h[o:o + n * n].reshape((n, n), order="F") for o, n in zip(self.off, self.n)]

    def unpack_sigma(self, sig):
        h = sig.detach().cpu().numpy()
        return [h[o:o + n] for o, n in zip(self.soff, self.n)]


def workspace_bytes(dtype, n):
    n = np.ascontiguousarray(n, dtype=np.int32)
    return int(_lib.lib().kog_sweep_workspace_size(_DT[dtype], len(n),
                                                   n.ctypes.data_as(ctypes.c_void_p)))


def kog_sweep_batch(packed: Packed, max_sweeps: int = 30, tol_factor: float = 1.0,
                    mode: str | int = "persistent", U=None, V=None, workspace=None,
                    sort: bool = False, ordering: str | int = "modulus"):
    """Run the sweep in place on packed.G.  Returns dict(G, U, V, sigma, sweeps).

    ``ordering``: "modulus" (1, the modified modulus strategy; the default: on the
    benchmark batches it needs 2 to 2.5 times fewer sweeps) or "round-robin" (0).
    ``U``/``V`` given => accumulate (continue from them).  ``sort`` => sigma in
    descending order with the columns of U and V permuted to match (kog_sweep_sort);
    G stays the iterate, so resume only from unsorted U and V."""
    L = _lib.lib()
    mode = MODES.get(mode, mode)
    ordering = ORDERINGS.get(ordering, ordering)
    G = packed.G
    dt = _DT[G.dtype]
    acc = U is not None
    if U is None:
        U = torch.empty_like(G)
        V = torch.empty_like(G)
    sigma = torch.empty(int(packed.n.sum()), dtype=G.dtype, device=G.device)
    sweeps = torch.empty(len(packed.n), dtype=torch.int32, device=G.device)
    need = workspace_bytes(G.dtype, packed.n)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device=G.device)
    wsp = workspace.data_ptr()
    pad = (-wsp) % 256
    n = np.ascontiguousarray(packed.n)
    off = np.ascontiguousarray(packed.off)
    cur = torch.cuda.current_stream()
    side = None
    stream = cur
    if mode == 2:
        side = _side_stream(G.device)
        side.wait_stream(cur)
        stream = side
    with torch.cuda.stream(stream):
        rc = L.kog_sweep_batch(dt, len(n), n.ctypes.data_as(ctypes.c_void_p),
                               off.ctypes.data_as(ctypes.c_void_p), G.data_ptr(), U.data_ptr(),
                               V.data_ptr(), sigma.data_ptr(), sweeps.data_ptr(), int(max_sweeps),
                               float(tol_factor), int(acc), int(mode), int(ordering), wsp + pad,
                               workspace.numel() - pad, stream.cuda_stream or None)
    _lib.check(rc, "kog_sweep_batch")
    if sort:
        with torch.cuda.stream(stream):
            rc = L.kog_sweep_sort(dt, len(n), n.ctypes.data_as(ctypes.c_void_p),
                                  off.ctypes.data_as(ctypes.c_void_p), U.data_ptr(),
                                  V.data_ptr(), sigma.data_ptr(), wsp + pad,
                                  workspace.numel() - pad, stream.cuda_stream or None)
        _lib.check(rc, "kog_sweep_sort")
    if side is not None:
        cur.wait_stream(side)
        for t in (G, U, V, sigma, sweeps, workspace):
            t.record_stream(side)
    return {"G": G, "U": U, "V": V, "sigma": sigma, "sweeps": sweeps, "workspace": workspace}


_SIDE = {}


def _side_stream(device):
    key = torch.device(device).index or 0
    if key not in _SIDE:
        _SIDE[key] = torch.cuda.Stream(device=device)   # default priority
    return _SIDE[key]


def sigma_grad(packed: Packed, U, V, dsigma, workspace=None):
    """dG = U diag(dsigma) V^T per matrix (the gradient of sum dsigma_i sigma_i).
    `workspace` may be the one kog_sweep_batch returned (it is large enough)."""
    L = _lib.lib()
    dG = torch.empty_like(U)
    need = workspace_bytes(U.dtype, packed.n)
    ws = workspace
    if ws is None or ws.numel() < need + 256:
        ws = torch.empty(need + 256, dtype=torch.uint8, device=U.device)
    pad = (-ws.data_ptr()) % 256
    n = np.ascontiguousarray(packed.n)
    off = np.ascontiguousarray(packed.off)
    rc = L.kog_sigma_grad(_DT[U.dtype], len(n), n.ctypes.data_as(ctypes.c_void_p),
                          off.ctypes.data_as(ctypes.c_void_p), U.data_ptr(), V.data_ptr(),
                          dsigma.data_ptr(), dG.data_ptr(), ws.data_ptr() + pad,
                          ws.numel() - pad, torch.cuda.current_stream().cuda_stream or None)
    _lib.check(rc, "kog_sigma_grad")
    return dG


class PackedRect:
    """m x n matrices (m >= n) packed column-major into one flat device tensor, with the
    n x n buffers (offsets roff) their triangular factors and V use."""

    def __init__(self, mats, dtype=None, device="cuda"):
        mats = [np.asarray(x) for x in mats]
        dtype = dtype or mats[0].dtype
        self.m = np.array([x.shape[0] for x in mats], dtype=np.int32)
        self.n = np.array([x.shape[1] for x in mats], dtype=np.int32)
        self.aoff = np.concatenate([[0], np.cumsum(self.m.astype(np.int64) * self.n)[:-1]]
                                   ).astype(np.int64)
        self.A = torch.from_numpy(np.concatenate([np.asarray(x, dtype=dtype).ravel(order="F")
                                                  for x in mats])).to(device)
        self.R = Packed([np.zeros((k, k), dtype) for k in self.n], dtype=dtype, device=device)
        self.roff = self.R.off
        self.A0 = self.A.clone()

    def reset(self):
        self.A.copy_(self.A0)


def svd_rect_device(pr: PackedRect, max_sweeps: int = 40, tol_factor: float = 1.0,
                    mode="persistent", ordering="modulus", sort: bool = True):
    """kog_qrcp_batch, the sweep on the triangular factors (kog_sweep_sort when ``sort``)
    and kog_qrcp_apply on a PackedRect (its A is overwritten by the reflectors).
    Returns dict(U, V, sigma, sweeps) of device tensors (U in A's layout, V in R's)."""
    L = _lib.lib()
    dev = pr.A.device
    ntot = int(pr.n.sum())
    tau = torch.empty(ntot, dtype=pr.A.dtype, device=dev)
    perm = torch.empty(ntot, dtype=torch.int32, device=dev)
    wsz = int(L.kog_rect_workspace_size(len(pr.m)))
    ws = torch.empty(wsz + 256, dtype=torch.uint8, device=dev)
    pad = (-ws.data_ptr()) % 256
    st = torch.cuda.current_stream().cuda_stream or None
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    dt = _DT[pr.A.dtype]
    m, n, aoff, roff = (np.ascontiguousarray(x) for x in (pr.m, pr.n, pr.aoff, pr.roff))
    rc = L.kog_qrcp_batch(dt, len(m), ptr(m), ptr(n), ptr(aoff), ptr(roff), pr.A.data_ptr(),
                          tau.data_ptr(), perm.data_ptr(), pr.R.G.data_ptr(),
                          ws.data_ptr() + pad, wsz, st)
    _lib.check(rc, "kog_qrcp_batch")
    out = kog_sweep_batch(pr.R, max_sweeps=max_sweeps, tol_factor=tol_factor, mode=mode,
                          sort=sort, ordering=ordering)
    U = torch.empty_like(pr.A)
    V = torch.empty_like(pr.R.G)
    rc = L.kog_qrcp_apply(dt, len(m), ptr(m), ptr(n), ptr(aoff), ptr(roff), pr.A.data_ptr(),
                          tau.data_ptr(), perm.data_ptr(), out["U"].data_ptr(),
                          out["V"].data_ptr(), U.data_ptr(), V.data_ptr(), ws.data_ptr() + pad,
                          wsz, st)
    _lib.check(rc, "kog_qrcp_apply")
    return {"U": U, "V": V, "sigma": out["sigma"], "sweeps": out["sweeps"]}


def svd_rect(mats, max_sweeps: int = 40, tol_factor: float = 1.0, mode="persistent",
             ordering="modulus", sort: bool = True, dtype=None, device="cuda"):
    """SVD of m x n matrices (Sect. 1) through svd_rect_device: G = U diag(sigma) V^T
    with U [m,k], V [n,k], k = min(m, n), which must be even.  A matrix with m < n is
    factored as G^T (the paper's advice) and its U and V exchanged.  Returns a list of
    (U, sigma, V) numpy triples and the sweep counts."""
    mats = [np.asarray(x) for x in mats]
    wide = [x.shape[0] < x.shape[1] for x in mats]
    mats = [x.T if w else x for x, w in zip(mats, wide)]
    pr = PackedRect(mats, dtype=dtype, device=device)
    out = svd_rect_device(pr, max_sweeps, tol_factor, mode, ordering, sort)
    Uh = out["U"].cpu().numpy()
    Vs = pr.R.unpack(out["V"])
    sig = pr.R.unpack_sigma(out["sigma"])
    res = [(Uh[o:o + mm * nn].reshape((mm, nn), order="F"), sig[k], Vs[k])
           for k, (o, mm, nn) in enumerate(zip(pr.aoff, pr.m, pr.n))]
    res = [(V, s_, U) if w else (U, s_, V) for (U, s_, V), w in zip(res, wide)]
    return res, out["sweeps"].cpu().numpy()


# knobs of the persistent sweep's tuning table (kog_sweep_set_tuning); none of them
# changes a bit of the results
KNOBS = {"block": 0, "chunk": 1, "two": 2, "inplace": 3, "rows": 4}


def set_tuning(dtype, bucket: int, block: int | None = None, **knobs):
    """Set entries of the tuning table for an order bucket (-1: every bucket):
    ``block`` and any of the KNOBS as keywords."""
    if block is not None:
        knobs["block"] = block
    for k, v in knobs.items():
        _lib.check(_lib.lib().kog_sweep_set_tuning(_DT[dtype], bucket, KNOBS[k], int(v)),
                   "kog_sweep_set_tuning")


def get_tuning(dtype, bucket: int) -> dict:
    L = _lib.lib()
    return {k: int(L.kog_sweep_get_tuning(_DT[dtype], bucket, v)) for k, v in KNOBS.items()}


def reset_tuning():
    _lib.check(_lib.lib().kog_sweep_reset_tuning(), "kog_sweep_reset_tuning")
