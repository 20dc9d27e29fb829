"""Pins of the oracle's rectangular path (Sect. 1: an m x n matrix, m > n, is first
reduced to a square triangular matrix by the QR factorization with column pivoting).

* the factorization against LAPACK's dgeqp3 (scipy.linalg.qr with pivoting, run as a
  library): the same column permutation (also on exact ties of the column norms: the
  first column wins) and the same R, signs included;
* Q (formed from the reflectors) orthogonal, G P = Q R, |r_kk| non-increasing;
* the whole SVD (QRCP, the sweep on R, U = Q [U_R; 0], V = P V_R): LAPACK's singular
  values, orthonormal U columns, orthogonal V, G = U Sigma V^T.
"""
import numpy as np
import pytest
import scipy.linalg as sl

DT = [np.float64, np.float32]


def _eps(dt):
    return 2.0 ** (-53 if dt == np.float64 else -24)


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("m,n", [(2, 2), (8, 4), (40, 10), (100, 64), (33, 32)])
def test_qrcp_matches_lapack(orc, dt, m, n):
    rng = np.random.default_rng(m * 100 + n)
    G = (rng.standard_normal((m, n)) * np.exp2(rng.integers(-4, 5, n))).astype(dt)
    A, tau, perm, R = orc.qrcp(G)
    Q2, R2, P2 = sl.qr(G.astype(np.float64), pivoting=True, mode="economic")
    assert np.array_equal(perm, P2)
    scale = np.linalg.norm(G.astype(np.float64))
    # the same reflector convention (beta = -sign(x0) ||x||): the same signs
    assert np.abs(R - R2).max() <= 8 * m * _eps(dt) * scale
    d = np.abs(np.diag(R.astype(np.float64)))
    assert np.all(d[:-1] >= d[1:] * (1 - 8 * m * _eps(dt)))
    # Q from the reflectors: U = Q [I; 0]
    Q, _ = orc.qapply(A, tau, perm, np.eye(n, dtype=dt), np.eye(n, dtype=dt))
    Qd = Q.astype(np.float64)
    assert np.abs(Qd.T @ Qd - np.eye(n)).max() <= 8 * m * _eps(dt)
    assert np.abs(Qd @ R.astype(np.float64) - G.astype(np.float64)[:, perm]).max() \
        <= 8 * m * _eps(dt) * scale
    assert np.all(np.tril(R, -1) == 0)


@pytest.mark.parametrize("dt", DT)
@pytest.mark.parametrize("m,n", [(4, 2), (64, 16), (130, 64), (65, 64)])
def test_rect_svd(orc, dt, m, n):
    rng = np.random.default_rng(7 * m + n)
    G = (rng.standard_normal((m, n)) * np.exp2(rng.integers(-3, 4, (m, n)))).astype(dt)
    U, s, V, sw = orc.svd_rect(G)
    assert sw > 0
    e = _eps(dt)
    Gd = G.astype(np.float64)
    ref = np.linalg.svd(Gd, compute_uv=False)
    got = np.sort(np.abs(s.astype(np.float64)))[::-1]
    assert np.abs(got - ref).max() <= 20 * m * e * ref[0]
    Ud, Vd = U.astype(np.float64), V.astype(np.float64)
    assert np.abs(Ud.T @ Ud - np.eye(n)).max() <= 20 * m * e
    assert np.abs(Vd.T @ Vd - np.eye(n)).max() <= 20 * n * e
    assert np.abs(Ud @ np.diag(s.astype(np.float64)) @ Vd.T - Gd).max() \
        <= 20 * m * e * np.linalg.norm(Gd)


@pytest.mark.parametrize("dt", DT)
def test_qrcp_ties_pick_the_first_column(orc, dt):
    rng = np.random.default_rng(11)
    G = rng.standard_normal((20, 6)).astype(dt)
    G[:, 1] *= 10
    G[:, 4] = G[:, 1]          # the two largest norms, exactly equal
    G[:, 5] = -G[:, 2]
    A, tau, perm, R = orc.qrcp(G)
    _, _, P2 = sl.qr(G.astype(np.float64), pivoting=True, mode="economic")
    assert perm[0] == P2[0]
    assert perm[0] == 1



@pytest.mark.parametrize("dtype,shift", [(np.float64, 700), (np.float64, -700),
                                         (np.float32, 90), (np.float32, -90)])
def test_qrcp_scaled_inputs(orc, dtype, shift):
    """Entries whose squares leave the normal range: the factorization of G 2^shift has
    the pivots of G's, R = 2^shift R(G) bit for bit (the scaling is exact), the same
    reflectors and tau, and agrees with LAPACK."""
    rng = np.random.default_rng(31)
    G = (rng.standard_normal((40, 12)) * np.exp2(rng.integers(-3, 4, 12))).astype(dtype)
    Gs = np.ldexp(G, shift).astype(dtype)
    A0, t0, p0, R0 = orc.qrcp(G)
    A1, t1, p1, R1 = orc.qrcp(Gs)
    assert np.all(np.isfinite(R1)) and np.array_equal(p0, p1)
    assert np.array_equal(R1, np.ldexp(R0, shift).astype(dtype))
    assert np.array_equal(np.tril(A1, -1), np.tril(A0, -1)) and np.array_equal(t1, t0)
    if dtype == np.float64:
        import scipy.linalg as sla

        Rl, P = sla.qr(Gs, mode="r", pivoting=True)
        assert np.array_equal(P, p1)
        scale = np.abs(Rl).max()
        assert np.abs(np.abs(np.diag(R1[:12, :12])) - np.abs(np.diag(Rl[:12, :12]))).max() <= 1e-13 * scale
