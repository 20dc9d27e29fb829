"""Python face of libksvd2: torch tensors in, torch tensors out.

Only argument marshalling happens here (dtype/device/contiguity checks, output
allocation, the current torch stream); every step of the method runs in the
HIP kernels behind the C ABI.
"""
from __future__ import annotations

import torch

from . import _lib

_DT = {torch.float32: 0, torch.float64: 1}


def _stream():
    return ctypes_ptr(torch.cuda.current_stream().cuda_stream)


def ctypes_ptr(v):
    return v if v is None else int(v)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _check_gpu(*ts):
    dt = None
    for t in ts:
        if t is None:
            continue
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise _lib.KSVD2Error("libksvd2 works on GPU tensors only (no CPU fallback)")
        if not t.is_contiguous():
            raise _lib.KSVD2Error("tensors must be contiguous")
        if t.dtype not in _DT:
            raise _lib.KSVD2Error(f"unsupported dtype {t.dtype}")
        if dt is None:
            dt = t.dtype
        elif t.dtype != dt:
            raise _lib.KSVD2Error("all floating-point tensors must share one dtype")
    return dt


def ksvd2_batch(g11, g21, g12, g22, plain: bool = True, out: dict | None = None,
                fast: bool = False):
    """The 2x2 SVD of a batch given as four planes (structure of arrays).

    Returns a dict of tensors: cu su cv sv f1 f2 (working precision), e1 e2 info
    (int32), and s1 s2 (plain sigma) when ``plain``.  ``fast`` selects the variant
    for a hypot that is not correctly rounded (ksvd2_batch_fast_*).  See
    include/ksvd2.h."""
    dt = _check_gpu(g11, g21, g12, g22)
    n = g11.numel()
    for g in (g21, g12, g22):
        if g.numel() != n:
            raise _lib.KSVD2Error("planes must have equal length")
    dev = g11.device
    if out is None:
        out = {k: torch.empty(n, dtype=dt, device=dev) for k in ("cu", "su", "cv", "sv", "f1", "f2")}
        for k in ("e1", "e2", "info"):
            out[k] = torch.empty(n, dtype=torch.int32, device=dev)
        if plain:
            out["s1"] = torch.empty(n, dtype=dt, device=dev)
            out["s2"] = torch.empty(n, dtype=dt, device=dev)
    L = _lib.lib()
    if fast:
        fn = L.ksvd2_batch_fast_f64 if dt == torch.float64 else L.ksvd2_batch_fast_f32
    else:
        fn = L.ksvd2_batch_f64 if dt == torch.float64 else L.ksvd2_batch_f32
    rc = fn(n, _ptr(g11), _ptr(g21), _ptr(g12), _ptr(g22), _ptr(out["cu"]), _ptr(out["su"]),
            _ptr(out["cv"]), _ptr(out["sv"]), _ptr(out["f1"]), _ptr(out["f2"]), _ptr(out["e1"]),
            _ptr(out["e2"]), _ptr(out["info"]), _ptr(out.get("s1")), _ptr(out.get("s2")),
            _stream())
    _lib.check(rc, "ksvd2_batch")
    return out


def svd2x2_raw(G, with_info: bool = False):
    """Forward in the autograd layout: G [B,2,2] -> (U [B,2,2], S [B,2], V [B,2,2])."""
    dt = _check_gpu(G)
    if G.dim() != 3 or G.shape[1:] != (2, 2):
        raise _lib.KSVD2Error("G must have shape [B,2,2]")
    B = G.shape[0]
    U = torch.empty_like(G)
    V = torch.empty_like(G)
    S = torch.empty((B, 2), dtype=dt, device=G.device)
    info = torch.empty(B, dtype=torch.int32, device=G.device) if with_info else None
    rc = _lib.lib().ksvd2_svd2x2(_DT[dt], B, _ptr(G), _ptr(U), _ptr(S), _ptr(V), _ptr(info),
                                 _stream())
    _lib.check(rc, "ksvd2_svd2x2")
    return (U, S, V, info) if with_info else (U, S, V)


def svd2x2_backward(U, S, V, dS=None, dU=None, dV=None, tau: float = 0.0):
    """The adjoint of G = U diag(S) V^T (layouts as svd2x2_raw); returns dG [B,2,2]."""
    dt = _check_gpu(U, S, V, dS, dU, dV)
    B = U.shape[0]
    dG = torch.empty_like(U)
    rc = _lib.lib().ksvd2_svd2x2_backward(_DT[dt], B, _ptr(U), _ptr(S), _ptr(V), _ptr(dS),
                                          _ptr(dU), _ptr(dV), _ptr(dG), float(tau), _stream())
    _lib.check(rc, "ksvd2_svd2x2_backward")
    return dG


def ksvd2_backward_soa(fwd: dict, ds1=None, ds2=None, dU=None, dV=None, tau: float = 0.0,
                       out=None):
    """The adjoint on the planes of ``ksvd2_batch(..., plain=True)``: ``fwd`` holds cu su
    cv sv info s1 s2; ds1, ds2 are planes; dU, dV are [4, B] tensors holding the entries
    (1,1), (2,1), (1,2), (2,2) of every matrix (each argument may be None: zero).
    Returns dG as a [4, B] tensor of the planes g11, g21, g12, g22 (or fills ``out``)."""
    for k in ("cu", "su", "cv", "sv", "info", "s1", "s2"):
        if fwd.get(k) is None:
            raise _lib.KSVD2Error(f"ksvd2_backward_soa: forward plane {k} missing "
                                  "(run ksvd2_batch with plain=True)")
    dt = _check_gpu(fwd["cu"], fwd["su"], fwd["cv"], fwd["sv"], fwd["s1"], fwd["s2"], ds1, ds2,
                    dU, dV, out)
    inf = fwd["info"]
    if not (inf.is_cuda and inf.is_contiguous() and inf.dtype == torch.int32):
        raise _lib.KSVD2Error("ksvd2_backward_soa: info must be a contiguous int32 GPU tensor")
    B = fwd["cu"].numel()
    for t in (dU, dV, out):
        if t is not None and tuple(t.shape) != (4, B):
            raise _lib.KSVD2Error("dU, dV and out must have shape [4, B]")
    for t in (ds1, ds2):
        if t is not None and t.numel() != B:
            raise _lib.KSVD2Error("ds1 and ds2 must have B elements")
    if out is None:
        out = torch.empty((4, B), dtype=dt, device=fwd["cu"].device)
    rc = _lib.lib().ksvd2_batch_backward(
        _DT[dt], B, _ptr(fwd["cu"]), _ptr(fwd["su"]), _ptr(fwd["cv"]), _ptr(fwd["sv"]),
        _ptr(fwd["info"]), _ptr(fwd["s1"]), _ptr(fwd["s2"]), _ptr(ds1), _ptr(ds2), _ptr(dU),
        _ptr(dV), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _ptr(out[3]), float(tau),
        _stream())
    _lib.check(rc, "ksvd2_batch_backward")
    return out


def hypot(x, y, fast: bool = False):
    """hypot on the device (elementwise): correctly rounded, or the fast variant's."""
    dt = _check_gpu(x, y)
    out = torch.empty_like(x)
    L = _lib.lib()
    fn = L.ksvd2_hypot_fast_batch if fast else L.ksvd2_hypot_batch
    rc = fn(_DT[dt], x.numel(), _ptr(x), _ptr(y), _ptr(out), _stream())
    _lib.check(rc, "ksvd2_hypot_batch")
    return out


def ksvd2c(G, with_pairs: bool = False):
    """Complex 2x2 SVD (Sect. 3.4): G [B,2,2] complex64/complex128 on the GPU ->
    (U [B,2,2], S [B,2] real, V [B,2,2]) with G = U diag(S) V^H; with ``with_pairs``
    also (f [B,2], e [B,2] int32, info [B] int32), sigma = f 2^e.  See ksvd2c_batch."""
    if not isinstance(G, torch.Tensor) or not G.is_cuda:
        raise _lib.KSVD2Error("ksvd2c: G must be a CUDA tensor (no CPU fallback)")
    if G.dtype not in (torch.complex64, torch.complex128):
        raise _lib.KSVD2Error("ksvd2c: G must be complex64 or complex128")
    if G.dim() != 3 or G.shape[1:] != (2, 2):
        raise _lib.KSVD2Error("ksvd2c: G must have shape [B,2,2]")
    G = G.contiguous()
    rt = torch.float64 if G.dtype == torch.complex128 else torch.float32
    B = G.shape[0]
    U = torch.empty_like(G)
    V = torch.empty_like(G)
    S = torch.empty((B, 2), dtype=rt, device=G.device)
    f = e = info = None
    if with_pairs:
        f = torch.empty((B, 2), dtype=rt, device=G.device)
        e = torch.empty((B, 2), dtype=torch.int32, device=G.device)
        info = torch.empty(B, dtype=torch.int32, device=G.device)
    rc = _lib.lib().ksvd2c_batch(1 if rt == torch.float64 else 0, B, _ptr(G), _ptr(U), _ptr(S),
                                 _ptr(V), _ptr(f), _ptr(e), _ptr(info), _stream())
    _lib.check(rc, "ksvd2c_batch")
    return (U, S, V, f, e, info) if with_pairs else (U, S, V)


class SVD2x2(torch.autograd.Function):
    """G [B,2,2] -> (U, S, V) with G = U diag(S) V^T; backward by the adjoint kernel.

    ``tau`` > 0 selects Lorentzian broadening of 1/(s1 - s2) in the backward pass
    (see include/ksvd2.h)."""

    @staticmethod
    def forward(ctx, G, tau: float = 0.0):
        U, S, V = svd2x2_raw(G.contiguous())
        ctx.save_for_backward(U, S, V)
        ctx.tau = tau
        return U, S, V

    @staticmethod
    def backward(ctx, dU, dS, dV):
        U, S, V = ctx.saved_tensors
        dU = None if dU is None else dU.contiguous()
        dS = None if dS is None else dS.contiguous()
        dV = None if dV is None else dV.contiguous()
        dG = svd2x2_backward(U, S, V, dS, dU, dV, ctx.tau)
        return dG, None


def svd2x2(G, tau: float = 0.0):
    """Differentiable batched 2x2 SVD (torch.autograd.Function)."""
    return SVD2x2.apply(G, tau)
