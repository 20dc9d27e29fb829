"""Seeded synthetic inputs for the batched 2x2 SVD, its adjoint and the sweep.

This module holds no arithmetic of the method: it only draws matrices.  It is
the one piece of code that both the GPU path (via the tests and the benchmark)
and the CPU oracle are fed from.  All generators use numpy's PCG64 with a fixed
seed, so every input is reproducible.

The recipes stand in for the paper's random test families (Sect. 4: entries
below one in magnitude from a seeded PRNG, and entries across the safe range
[mu, nu/4]); sizes and value distributions follow the workload table of the
project's design notes:

* ``forward_small``   65,536 float64 matrices, entries +-m 2^e with m uniform on
  the p-bit grid of [1,2), e uniform integer in [-20,20]; 5% carry a zero
  pattern (upper / lower triangular, diagonal, one zero, all zeros).
* ``forward_sweep``   2^24 matrices, float64 with e in [-1000,1000] or float32
  with e in [-120,120]; 10% upper triangular; 1% near-singular
  (row2 = RN(row1 (1 + 2^-k)), k uniform in [1,50]).
* ``diff_batch``      2^22 matrices, N(0,1) 2^e with e in [-10,10]; 1% with
  sigma1/sigma2 - 1 < 1e-6 and 1% rank-deficient; upstream gradients N(0,1).
* ``sweep_uniform``   256 matrices of order 256, N(0,1) with column j scaled by
  2^(-j/8).
* ``sweep_uneven``    1,000 matrices, order uniform even in [16,512],
  N(0,1) 2^e with e in [-30,30].
* ``special_set``     every zero pattern x signs x magnitudes from a table of
  edge values (zeros of both signs, subnormals, mu, nu, ties).

SoA layout: a batch is four planes ``g11, g21, g12, g22`` (column-major order
of the 2x2 matrix), each a contiguous array of length B.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "soa_from_mats", "mats_from_soa", "signed_pow2_entries", "forward_small", "forward_sweep",
    "diff_batch", "sweep_uniform", "sweep_uneven", "special_set",
]


def _p(dtype) -> int:
    return 53 if np.dtype(dtype) == np.float64 else 24


def soa_from_mats(G: np.ndarray):
    """[B,2,2] (row-major 2x2) -> (g11, g21, g12, g22) contiguous planes."""
    G = np.asarray(G)
    return tuple(np.ascontiguousarray(G[:, i, j]) for (i, j) in ((0, 0), (1, 0), (0, 1), (1, 1)))


def mats_from_soa(g11, g21, g12, g22) -> np.ndarray:
    B = len(g11)
    G = np.empty((B, 2, 2), dtype=np.asarray(g11).dtype)
    G[:, 0, 0], G[:, 1, 0], G[:, 0, 1], G[:, 1, 1] = g11, g21, g12, g22
    return G


def signed_pow2_entries(rng, shape, emin, emax, dtype):
    """+-m 2^e, m = 1 + k 2^(1-p) with k uniform in [0, 2^(p-1)), e uniform in [emin, emax]."""
    p = _p(dtype)
    k = rng.integers(0, 2 ** (p - 1), size=shape, dtype=np.int64)
    m = 1.0 + k.astype(np.float64) * 2.0 ** (1 - p)  # exact in float64 for p <= 53
    e = rng.integers(emin, emax + 1, size=shape)
    s = np.where(rng.random(shape) < 0.5, -1.0, 1.0)
    if np.dtype(dtype) == np.float64:
        return s * np.ldexp(m, e)
    # float32: m has 24 bits and the exponent range is inside float32's normal range
    return (s * np.ldexp(m, e)).astype(np.float32)


def forward_small(seed: int = 1, B: int = 65536):
    """Config: plain forward, 65,536 float64 matrices with 5% zero patterns."""
    rng = np.random.default_rng(seed)
    G = signed_pow2_entries(rng, (B, 2, 2), -20, 20, np.float64)
    nz = int(round(0.05 * B))
    idx = rng.choice(B, size=nz, replace=False)
    kind = rng.integers(0, 5, size=nz)
    for i, k in zip(idx, kind):
        if k == 0:      # upper triangular
            G[i, 1, 0] = 0.0
        elif k == 1:    # lower triangular
            G[i, 0, 1] = 0.0
        elif k == 2:    # diagonal
            G[i, 1, 0] = 0.0
            G[i, 0, 1] = 0.0
        elif k == 3:    # a single zero at a uniform position
            pos = rng.integers(0, 4)
            G[i, pos // 2, pos % 2] = 0.0
        else:           # all zeros
            G[i] = 0.0
    return soa_from_mats(G)


def forward_sweep(dtype=np.float64, seed=None, B: int = 1 << 24, with_labels: bool = False):
    """Config: accuracy/throughput sweep.  float64: e in [-1000,1000] (seed 2);
    float32: e in [-120,120] (seed 3).  10% upper triangular, 1% near-singular.
    with_labels: also return the family of each matrix (0 general, 1 upper
    triangular, 2 near-singular)."""
    f64 = np.dtype(dtype) == np.float64
    if seed is None:
        seed = 2 if f64 else 3
    rng = np.random.default_rng(seed)
    emax = 1000 if f64 else 120
    G = signed_pow2_entries(rng, (B, 2, 2), -emax, emax, dtype)
    u = rng.random(B)
    tri = u < 0.10
    G[tri, 1, 0] = 0
    near = (u >= 0.10) & (u < 0.11)
    ni = np.nonzero(near)[0]
    k = rng.integers(1, 51, size=ni.size)
    delta = np.ldexp(np.ones(ni.size), -k).astype(dtype)
    for j in range(2):
        r1 = G[ni, 0, j]
        # RN(g (1 + delta)): g*delta is exact (a power-of-two scaling), one rounding in the sum
        G[ni, 1, j] = r1 + r1 * delta
    if with_labels:
        lab = np.zeros(B, np.int8)
        lab[tri] = 1
        lab[near] = 2
        return soa_from_mats(G), lab
    return soa_from_mats(G)


def diff_batch(dtype=np.float64, seed=None, B: int = 1 << 22):
    """Config: differentiable batch.  Returns (G[B,2,2], dS[B,2], dU[B,2,2], dV[B,2,2],
    labels) with labels 0 general, 1 near-degenerate (sigma1/sigma2 - 1 < 1e-6),
    2 rank-deficient.  The first 4,096 matrices hold a stratified mix of all three."""
    f64 = np.dtype(dtype) == np.float64
    if seed is None:
        seed = 4 if f64 else 5
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((B, 2, 2)) * np.ldexp(1.0, rng.integers(-10, 11, (B, 2, 2)))
    labels = np.zeros(B, np.int8)
    u = rng.random(B)
    labels[u < 0.01] = 1
    labels[(u >= 0.01) & (u < 0.02)] = 2
    # stratify the first 4,096: 1/8 near-degenerate, 1/8 rank-deficient
    head = min(B, 4096)
    labels[:head] = 0
    labels[0:head:8] = 1
    labels[1:head:8] = 2
    nd = np.nonzero(labels == 1)[0]
    a = rng.random(nd.size) * 2 * np.pi
    b = rng.random(nd.size) * 2 * np.pi
    sig = np.ldexp(1.0, rng.integers(-10, 11, nd.size)) * (1 + rng.random(nd.size))
    gam = 1e-9 + rng.random(nd.size) * (1e-6 - 1e-9)
    ca, sa, cb, sb = np.cos(a), np.sin(a), np.cos(b), np.sin(b)
    s2 = sig * (1 - gam)
    # U_a diag(sig, s2) V_b^T
    G[nd, 0, 0] = ca * sig * cb + (-sa) * s2 * (-sb)
    G[nd, 0, 1] = ca * sig * sb + (-sa) * s2 * cb
    G[nd, 1, 0] = sa * sig * cb + ca * s2 * (-sb)
    G[nd, 1, 1] = sa * sig * sb + ca * s2 * cb
    rd = np.nonzero(labels == 2)[0]
    fac = np.where(rng.random(rd.size) < 0.5, -1.0, 1.0) * np.ldexp(1.0, rng.integers(-3, 4, rd.size))
    G[rd, 1, 0] = fac * G[rd, 0, 0]
    G[rd, 1, 1] = fac * G[rd, 0, 1]
    G = G.astype(dtype)
    rng2 = np.random.default_rng(seed + 100)
    dS = rng2.standard_normal((B, 2)).astype(dtype)
    dU = rng2.standard_normal((B, 2, 2)).astype(dtype)
    dV = rng2.standard_normal((B, 2, 2)).astype(dtype)
    return G, dS, dU, dV, labels


def sweep_uniform(seed: int = 6, nmat: int = 256, n: int = 256, dtype=np.float64):
    """Config: 256 matrices of order 256, G_ij = N(0,1) 2^(-j/8) (j 0-based column),
    returned as [nmat, n, n] arrays in column-major element order per matrix
    (i.e. element (i, j) at flat index i + j n)."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((nmat, n, n))
    scale = np.exp2(-np.arange(n) / 8.0)
    G = Z * scale[None, None, :]
    return [np.asfortranarray(G[k].astype(dtype)) for k in range(nmat)]


def sweep_uneven(seed: int = 7, nmat: int = 1000, dtype=np.float64, nmin: int = 16,
                 nmax: int = 512):
    """Config: 1,000 matrices, n uniform even in [16,512], N(0,1) 2^e with e in [-30,30]."""
    rng = np.random.default_rng(seed)
    ns = 2 * rng.integers(nmin // 2, nmax // 2 + 1, size=nmat)
    mats = []
    for n in ns:
        G = rng.standard_normal((n, n)) * np.ldexp(1.0, rng.integers(-30, 31, (n, n)))
        mats.append(np.asfortranarray(G.astype(dtype)))
    return mats


def _edge_magnitudes(dtype):
    f = np.finfo(dtype)
    tiny = np.array(f.smallest_subnormal, dtype)
    one = np.array(1, dtype)
    mags = [one, one + f.eps, 3 * one, np.array(0.75, dtype), f.tiny, tiny, 3 * tiny,
            f.max, f.max / 4, np.nextafter(f.tiny, 0).astype(dtype),
            np.array(2.0 ** (f.maxexp // 2), dtype), np.array(2.0 ** (f.minexp // 2), dtype),
            np.array(1.4142135623730951, dtype)]
    return np.array(mags, dtype=dtype)


def special_set(dtype=np.float64, seed: int = 11, per_type: int = 4096):
    """Every zero pattern t = 0..15, signed zeros, and nonzeros drawn from a table of edge
    magnitudes (1, 1+eps, 3, 0.75, mu, the smallest subnormal, nu, nu/4, ...) or random
    values, so that ties, equal magnitudes and extreme scalings all occur."""
    rng = np.random.default_rng(seed)
    mags = _edge_magnitudes(dtype)
    out = []
    for t in range(16):
        G = np.empty((per_type, 4), dtype)
        for k in range(4):
            nzk = (t >> k) & 1
            if nzk:
                pick = rng.integers(0, len(mags) + 2, per_type)
                vals = np.where(pick < len(mags), mags[np.minimum(pick, len(mags) - 1)],
                                signed_pow2_entries(rng, per_type, -30, 30, dtype))
                sgn = np.where(rng.random(per_type) < 0.5, -1, 1).astype(dtype)
                G[:, k] = (sgn * vals).astype(dtype)
            else:
                G[:, k] = np.where(rng.random(per_type) < 0.5, -0.0, 0.0).astype(dtype)
        out.append(G)
    G = np.concatenate(out)
    # plane order: g11, g21, g12, g22 <-> bits 0, 1, 2, 3 of t
    return tuple(np.ascontiguousarray(G[:, k]) for k in range(4))


def complex_batch(dtype=np.complex128, seed: int = 8, B: int = 1 << 22, emax=None):
    """Complex 2x2 matrices [B,2,2]: real and imaginary parts each +-m 2^e with e
    uniform in [-emax, emax] (default 20) and m on the p-bit grid; 10% upper
    triangular, 5% with one zero part per element (purely real or imaginary elements),
    2% of each single-column / single-row / diagonal pattern, 1% purely real and 1%
    purely imaginary matrices."""
    rt = np.float64 if np.dtype(dtype) == np.complex128 else np.float32
    rng = np.random.default_rng(seed)
    if emax is None:
        emax = 20
    re = signed_pow2_entries(rng, (B, 2, 2), -emax, emax, rt)
    im = signed_pow2_entries(rng, (B, 2, 2), -emax, emax, rt)
    u = rng.random(B)
    tri = u < 0.10
    re[tri, 1, 0] = 0
    im[tri, 1, 0] = 0
    mixed = (u >= 0.10) & (u < 0.15)
    zr = mixed[:, None, None] & (rng.random((B, 2, 2)) < 0.5)
    re[zr] = 0
    zi = mixed[:, None, None] & ~zr
    im[zi] = 0
    col = (u >= 0.15) & (u < 0.17)
    re[col, :, 1] = 0
    im[col, :, 1] = 0
    row = (u >= 0.17) & (u < 0.19)
    re[row, 1, :] = 0
    im[row, 1, :] = 0
    dia = (u >= 0.19) & (u < 0.21)
    re[dia, 0, 1] = re[dia, 1, 0] = 0
    im[dia, 0, 1] = im[dia, 1, 0] = 0
    im[(u >= 0.21) & (u < 0.22)] = 0
    re[(u >= 0.22) & (u < 0.23)] = 0
    G = np.empty((B, 2, 2), dtype)
    G.real = re
    G.imag = im
    return G


def complex_special_set(dtype=np.complex128, seed: int = 12, per_type: int = 1024):
    """Every zero pattern of the complex elements x the edge magnitudes of the real special
    set in either part (the other part zero, an edge value or a random value)."""
    rt = np.float64 if np.dtype(dtype) == np.complex128 else np.float32
    rng = np.random.default_rng(seed)
    mags = _edge_magnitudes(rt)
    out = []
    for t in range(16):
        G = np.zeros((per_type, 2, 2), dtype)
        for k, (i, j) in enumerate(((0, 0), (1, 0), (0, 1), (1, 1))):
            if not (t >> k) & 1:
                continue
            parts = []
            for _ in range(2):
                pick = rng.integers(0, len(mags) + 3, per_type)
                vals = np.where(pick < len(mags), mags[np.minimum(pick, len(mags) - 1)],
                                signed_pow2_entries(rng, per_type, -30, 30, rt))
                vals = np.where(pick == len(mags) + 2, 0, vals)
                sgn = np.where(rng.random(per_type) < 0.5, -1, 1)
                parts.append((sgn * vals).astype(rt))
            re, im = parts
            both0 = (re == 0) & (im == 0)
            re = np.where(both0, mags[0], re).astype(rt)
            G[:, i, j].real = re
            G[:, i, j].imag = im
        out.append(G)
    return np.concatenate(out)


def rect_batch(seed: int = 9, nmat: int = 256, m: int = 512, n: int = 256, dtype=np.float64):
    """Tall m x n matrices: N(0,1) entries with column j scaled by 2^(-j/8) (the uniform
    sweep workload's grading), column-major arrays."""
    rng = np.random.default_rng(seed)
    scale = np.exp2(-np.arange(n) / 8.0)
    return [np.asfortranarray((rng.standard_normal((m, n)) * scale).astype(dtype))
            for _ in range(nmat)]
