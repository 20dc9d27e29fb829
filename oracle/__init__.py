"""CPU oracle for the enhanced Kogbetliantz SVD of order two (arXiv 2407.13116).

TEST INFRASTRUCTURE ONLY.  This package is the independent reference that the
GPU library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the GPU library and
its Python binding never do, and the two share no code.

``liboracle.so`` is built from ``ksvd2_oracle.cpp`` with contraction disabled,
so every fused multiply-add in it is an explicit ``fma`` call.  The wrappers
below only marshal numpy arrays; the arithmetic is in the C++ file, except the
SVD adjoint (``svd2_backward``), which is the closed-form formula written out in
numpy float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ksvd2_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

CXXFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
            "-shared"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (contraction off, IEEE semantics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["g++", *CXXFLAGS, _SRC, "-o", tmp], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        d, f, i64, i32, p = (ctypes.c_double, ctypes.c_float, ctypes.c_int64, ctypes.c_int,
                             ctypes.c_void_p)
        L.orc_hypot_f64.restype = d
        L.orc_hypot_f64.argtypes = [d, d]
        L.orc_hypot_f32.restype = f
        L.orc_hypot_f32.argtypes = [f, f]
        for name in ("orc_hypot_batch_f64", "orc_hypot_batch_f32", "orc_hypot_fast_batch_f64",
                     "orc_hypot_fast_batch_f32"):
            getattr(L, name).argtypes = [i64, p, p, p]
        L.orc_ef_op_f64.argtypes = [i32, d, d, ctypes.POINTER(i32), ctypes.POINTER(d)]
        L.orc_ef_op_f32.argtypes = [i32, f, f, ctypes.POINTER(i32), ctypes.POINTER(f)]
        L.orc_ext_f64.restype = d
        L.orc_ext_f64.argtypes = [d, d, d, d, i32, d]
        L.orc_ext_f32.restype = f
        L.orc_ext_f32.argtypes = [f, f, f, f, i32, f]
        for name in ("orc_ksvd2_f64", "orc_ksvd2_f32", "orc_ksvd2_fast_f64",
                     "orc_ksvd2_fast_f32"):
            fn = getattr(L, name)
            fn.restype = i32
            fn.argtypes = [i64] + [p] * 15 + [i32]
        L.orc_urv15_f64.argtypes = [d, d, d, d, ctypes.POINTER(d), ctypes.POINTER(i32)]
        L.orc_urv15_f32.argtypes = [f, f, f, f, ctypes.POINTER(f), ctypes.POINTER(i32)]
        for name in ("orc_kog_sweep_f64", "orc_kog_sweep_f32"):
            fn = getattr(L, name)
            fn.restype = i32
            fn.argtypes = [i32, p, p, p, i32, d, i32, i32, ctypes.POINTER(i32)]
        L.orc_step_pairs.argtypes = [i32, i32, i32, p]
        L.orc_dynamic_pairs_f64.argtypes = [i32, p, p]
        for t in ("f64", "f32"):
            getattr(L, "orc_qrcp_" + t).argtypes = [i32, i32, p, p, p, p]
            getattr(L, "orc_qapply_" + t).argtypes = [i32, i32, p, p, p, p, p, p, p]
        for name in ("orc_ksvd2c_f64", "orc_ksvd2c_f32"):
            getattr(L, name).argtypes = [i64, p, p, p, p, p, p, p, i32]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dt(dtype):
    dtype = np.dtype(dtype)
    if dtype == np.float64:
        return "f64"
    if dtype == np.float32:
        return "f32"
    raise TypeError(f"unsupported dtype {dtype}")


def hypot(x, y, fast: bool = False):
    """hypot, elementwise (float64 or float32 arrays): correctly rounded, or (``fast``)
    the variant hi * sqrt(fma(r, r, 1)), r = lo / hi."""
    x = np.ascontiguousarray(x)
    y = np.ascontiguousarray(y, dtype=x.dtype)
    out = np.empty_like(x)
    kind = "orc_hypot_fast_batch_" if fast else "orc_hypot_batch_"
    getattr(lib(), kind + _dt(x.dtype))(x.size, _ptr(x), _ptr(y), _ptr(out))
    return out


def ef_op(op: str, x, y, dtype=np.float64):
    """One (e,f) operation: 'plus' (x (+) y), 'minus' (x (-) y), 'mul' (N(x) (.) N(y)),
    'div' (N(x) (/) N(y)).  Returns (e, f)."""
    code = {"plus": 0, "minus": 1, "mul": 2, "div": 3}[op]
    e = ctypes.c_int()
    if np.dtype(dtype) == np.float64:
        f = ctypes.c_double()
        lib().orc_ef_op_f64(code, float(x), float(y), ctypes.byref(e), ctypes.byref(f))
        return e.value, float(f.value)
    f = ctypes.c_float()
    lib().orc_ef_op_f32(code, float(x), float(y), ctypes.byref(e), ctypes.byref(f))
    return e.value, np.float32(f.value)


def ext(x1, y1, x2, y2, minus, d, dtype=np.float64):
    """fl(FL(FL(x1*y1 +- x2*y2)/d)) of eq. (EXT); T = double-word (f64) or binary64 (f32)."""
    if np.dtype(dtype) == np.float64:
        return lib().orc_ext_f64(x1, y1, x2, y2, int(minus), d)
    return np.float32(lib().orc_ext_f32(x1, y1, x2, y2, int(minus), d))


def urv15(g11, g21, g12, g22, dtype=np.float64):
    """The URV factorisation of one prescaled type-15 matrix: returns
    (r11, r12, r22, tan_theta, exact_tan, ext_used), r12 and r22 signed."""
    if np.dtype(dtype) == np.float64:
        out = (ctypes.c_double * 4)()
        fl = ctypes.c_int()
        lib().orc_urv15_f64(g11, g21, g12, g22, out, ctypes.byref(fl))
        vals = [float(v) for v in out]
    else:
        out = (ctypes.c_float * 4)()
        fl = ctypes.c_int()
        lib().orc_urv15_f32(g11, g21, g12, g22, out, ctypes.byref(fl))
        vals = [np.float32(v) for v in out]
    return (*vals, bool(fl.value & 1), bool(fl.value & 2))


def ksvd2(g11, g21, g12, g22, nthreads: int = 0, plain: bool = True, fast: bool = False):
    """Batched 2x2 SVD, SoA planes in, dict of SoA planes out (``fast``: the variant
    for a hypot that is not correctly rounded, Algorithm tf).

    Keys: cu su cv sv (U = [cu, -dU su; su, dU cu], likewise V, with dU/dV from the
    info bits 8/9), f1 f2 e1 e2 (sigma_i = f_i 2^e_i), info, and s1 s2 (sigma as
    plain floating-point values) when ``plain``."""
    g11 = np.ascontiguousarray(g11)
    dt = g11.dtype
    g21, g12, g22 = (np.ascontiguousarray(a, dtype=dt) for a in (g21, g12, g22))
    n = g11.size
    out = {k: np.empty(n, dt) for k in ("cu", "su", "cv", "sv", "f1", "f2")}
    for k in ("e1", "e2", "info"):
        out[k] = np.empty(n, np.int32)
    if plain:
        out["s1"] = np.empty(n, dt)
        out["s2"] = np.empty(n, dt)
    fn = getattr(lib(), ("orc_ksvd2_fast_" if fast else "orc_ksvd2_") + _dt(dt))
    bad = fn(n, _ptr(g11), _ptr(g21), _ptr(g12), _ptr(g22), _ptr(out["cu"]), _ptr(out["su"]),
             _ptr(out["cv"]), _ptr(out["sv"]), _ptr(out["f1"]), _ptr(out["f2"]),
             _ptr(out["e1"]), _ptr(out["e2"]), _ptr(out["info"]),
             _ptr(out["s1"]) if plain else None, _ptr(out["s2"]) if plain else None,
             int(nthreads))
    if bad:
        raise AssertionError(f"oracle: {bad} results with U or V not of the compact form")
    return out


def full_uv(out):
    """Expand the compact (c, s, det) outputs into U[B,2,2], V[B,2,2] (float64)."""
    info = out["info"].astype(np.int64)
    res = []
    for c, s, bit in (("cu", "su", 8), ("cv", "sv", 9)):
        cc = out[c].astype(np.float64)
        ss = out[s].astype(np.float64)
        d = np.where((info >> bit) & 1, -1.0, 1.0)
        M = np.empty(cc.shape + (2, 2))
        M[:, 0, 0] = cc
        M[:, 1, 0] = ss
        M[:, 0, 1] = -d * ss
        M[:, 1, 1] = d * cc
        res.append(M)
    return res[0], res[1]


def kog_sweep(G, max_sweeps: int = 30, tol_factor: float = 1.0, U=None, V=None,
              ordering: int = 1):
    """Two-sided Kogbetliantz iteration on one n x n matrix (parallel ordering 1 =
    modified modulus, the default, or 0 = round-robin).  G is taken column-major (pass a
    Fortran-ordered or transposed array); returns (G_out, U, V, status, sweeps) with
    the arrays column-major.  tol_factor < 0 disables the stopping test (exactly
    max_sweeps sweeps)."""
    G = np.array(G, order="F", copy=True)
    n = G.shape[0]
    dt = G.dtype
    acc = U is not None
    U = np.array(U, order="F", copy=True) if acc else np.empty((n, n), dt, order="F")
    V = np.array(V, order="F", copy=True) if acc else np.empty((n, n), dt, order="F")
    sw = ctypes.c_int()
    fn = getattr(lib(), "orc_kog_sweep_" + _dt(dt))
    st = fn(n, _ptr(G), _ptr(U), _ptr(V), int(max_sweeps), float(tol_factor), int(acc),
            int(ordering), ctypes.byref(sw))
    return G, U, V, st, sw.value


def ksvd2c(G, nthreads: int = 0):
    """Complex 2x2 SVD (Sect. 3.4) of G [B,2,2] (complex128 or complex64): returns dict
    U, V [B,2,2] complex (G = U diag(S) V^H), S [B,2] real, f [B,2], e [B,2] (sigma =
    f 2^e), info [B]."""
    G = np.ascontiguousarray(G)
    if G.dtype == np.complex128:
        rt = np.float64
    elif G.dtype == np.complex64:
        rt = np.float32
    else:
        raise TypeError(f"unsupported dtype {G.dtype}")
    B = G.shape[0]
    U = np.empty((B, 2, 2), G.dtype)
    V = np.empty((B, 2, 2), G.dtype)
    S = np.empty((B, 2), rt)
    f = np.empty((B, 2), rt)
    e = np.empty((B, 2), np.int32)
    info = np.empty(B, np.int32)
    fn = getattr(lib(), "orc_ksvd2c_" + _dt(rt))
    fn(B, _ptr(G), _ptr(U), _ptr(S), _ptr(V), _ptr(f), _ptr(e), _ptr(info), int(nthreads))
    return {"U": U, "V": V, "S": S, "f": f, "e": e, "info": info}


def qrcp(G):
    """QR with column pivoting of an m x n matrix (m >= n), Householder form:
    returns (A, tau, perm, R) with A holding the reflectors below the diagonal and R on
    and above (column-major), G[:, perm] = Q R, R the n x n triangular factor."""
    A = np.array(G, order="F", copy=True)
    m, n = A.shape
    tau = np.empty(n, A.dtype)
    perm = np.empty(n, np.int32)
    Rsq = np.empty((n, n), A.dtype, order="F")
    getattr(lib(), "orc_qrcp_" + _dt(A.dtype))(m, n, _ptr(A), _ptr(tau), _ptr(perm), _ptr(Rsq))
    return A, tau, perm, Rsq


def qapply(A, tau, perm, UR, VR):
    """U = Q [U_R; 0] (m x n) and V = P V_R from qrcp's output and the SVD of R."""
    m, n = A.shape
    A = np.asfortranarray(A)
    UR = np.asfortranarray(UR, dtype=A.dtype)
    VR = np.asfortranarray(VR, dtype=A.dtype)
    U = np.empty((m, n), A.dtype, order="F")
    V = np.empty((n, n), A.dtype, order="F")
    getattr(lib(), "orc_qapply_" + _dt(A.dtype))(m, n, _ptr(A), _ptr(np.ascontiguousarray(tau)),
                                                _ptr(np.ascontiguousarray(perm, np.int32)),
                                                _ptr(UR), _ptr(VR), _ptr(U), _ptr(V))
    return U, V


def svd_rect(G, max_sweeps: int = 40, tol_factor: float = 1.0, ordering: int = 1):
    """SVD of an m x n matrix (m >= n, n even): QR with column pivoting, the sweep on
    R, then U = Q [U_R; 0], V = P V_R.  Returns (U, sigma, V, sweeps), sigma unsorted
    as the sweep leaves it."""
    A, tau, perm, Rsq = qrcp(G)
    Gk, UR, VR, st, sw = kog_sweep(Rsq, max_sweeps=max_sweeps, tol_factor=tol_factor,
                                   ordering=ordering)
    U, V = qapply(A, tau, perm, UR, VR)
    return U, np.diag(Gk).copy(), V, (sw if st == 0 else -sw)


def step_pairs(ordering: int, n: int, k: int):
    """The n/2 pivot pairs (i < j) of step k of a sweep, as an int array [n/2, 2]."""
    out = np.empty((n // 2, 2), np.int32)
    lib().orc_step_pairs(int(ordering), int(n), int(k), _ptr(out))
    return out


def dynamic_pairs(G):
    """The pivot pairs the dynamic ordering takes for the square matrix G (float64, its
    own weights w_ij = g_ij^2 + g_ji^2), in the order the greedy matching took them, as
    an int array [n/2, 2] with i < j."""
    G = np.asfortranarray(G, dtype=np.float64)
    n = G.shape[0]
    out = np.empty((n // 2, 2), np.int32)
    lib().orc_dynamic_pairs_f64(int(n), _ptr(G), _ptr(out))
    return out


def svd2_backward(U, S, V, dS=None, dU=None, dV=None, tau: float = 0.0):
    """Adjoint of G = U diag(S) V^T for 2x2 matrices, float64, batched [B,2,2].

    With J = U^T dU and K = V^T dV, a = J12 - J21, b = K12 - K21, p = (a+b)/2,
    q = (a-b)/2, the core is M12 = -p/(s1-s2) + q/(s1+s2),
    M21 = -p/(s1-s2) - q/(s1+s2), and dG = U [[dS1, M12], [M21, dS2]] V^T
    (the square-matrix SVD adjoint with F_ij = 1/(s_j^2 - s_i^2), written out for
    order two).  Degenerate handling: 1/(s1-s2) becomes (s1-s2)/((s1-s2)^2+eta^2)
    with eta = tau*s1 when tau > 0; with tau = 0 the p-term is dropped when
    s1 - s2 == 0; the q-term is dropped when s1 + s2 == 0."""
    U = np.asarray(U, np.float64)
    V = np.asarray(V, np.float64)
    S = np.asarray(S, np.float64)
    B = U.shape[0]
    dS = np.zeros((B, 2)) if dS is None else np.asarray(dS, np.float64)
    dU = np.zeros((B, 2, 2)) if dU is None else np.asarray(dU, np.float64)
    dV = np.zeros((B, 2, 2)) if dV is None else np.asarray(dV, np.float64)
    J = np.einsum("bki,bkj->bij", U, dU)
    K = np.einsum("bki,bkj->bij", V, dV)
    a = J[:, 0, 1] - J[:, 1, 0]
    b = K[:, 0, 1] - K[:, 1, 0]
    p = 0.5 * (a + b)
    q = 0.5 * (a - b)
    s1, s2 = S[:, 0], S[:, 1]
    dm = s1 - s2
    sm = s1 + s2
    with np.errstate(divide="ignore", invalid="ignore"):
        if tau > 0:
            eta = tau * s1
            inv_dm = np.where(dm ** 2 + eta ** 2 > 0, dm / (dm ** 2 + eta ** 2), 0.0)
        else:
            inv_dm = np.where(dm != 0, 1.0 / dm, 0.0)
        inv_sm = np.where(sm != 0, 1.0 / sm, 0.0)
    M = np.zeros((B, 2, 2))
    M[:, 0, 0] = dS[:, 0]
    M[:, 1, 1] = dS[:, 1]
    M[:, 0, 1] = -p * inv_dm + q * inv_sm
    M[:, 1, 0] = -p * inv_dm - q * inv_sm
    return np.einsum("bij,bjk,blk->bil", U, M, V)
