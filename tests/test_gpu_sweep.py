"""GPU parity of the batched Kogbetliantz sweep.

* With a fixed number of sweeps (stopping test off): G, U, V and sigma bit for bit equal
  to the oracle's sweep, for every execution mode (plain per-step launches, persistent,
  hipGraph), on an uneven batch (orders 2 .. 66, both precisions), and on orders 130 ..
  520 whose deferred U/V update spans several LDS row tiles and pivot passes.
* Converged runs: the three modes bitwise identical to each other; sigma against LAPACK,
  orthogonality of U and V, reconstruction, the off-diagonal stopping test.
* The uniform-size workload at full size (256 matrices of order 256, FP64) and the uneven
  one (1,000 orders 16..512, FP64 and FP32) in the launch configuration the benchmark
  times; sampled matrices recomputed by the oracle with the same number of sweeps, bit for
  bit.
* The sigma gradient dG = U diag(dsigma) V^T: against float64 numpy, against central
  differences of sorted sigma through the GPU sweep, and the contraction alone on general
  U and V of orders 1..300 (ragged tiles, several matrices per XCD) within its rounding
  bound.
* Resuming (accumulate): 1 + 1 sweeps equal 2 sweeps bitwise; edge cases (order 2,
  diagonal and zero matrices).
* Orderings: every case above runs the default modified modulus ordering; the
  round-robin ordering bit for bit against the oracle's sweep with that ordering, every
  mode, orders 2 .. 260 (several U/V tiles); converged runs of both orderings reach
  LAPACK's singular values.
"""
import numpy as np
import pytest

from paper_2407_13116_amd import inputs

pytestmark = pytest.mark.gpu
MODES = ["plain", "persistent", "graph"]
_LARGE_REF = {}


def _mats(rng, ns, dtype, emax=3):
    return [np.asfortranarray((rng.standard_normal((n, n)) *
                               np.exp2(rng.integers(-emax, emax + 1, (n, n)))).astype(dtype))
            for n in ns]


def _run(mats, dtype, mode, max_sweeps, tolf, ordering="modulus"):
    import torch

    from paper_2407_13116_amd import sweep as sw

    p = sw.Packed(mats, dtype=dtype)
    out = sw.kog_sweep_batch(p, max_sweeps=max_sweeps, tol_factor=tolf, mode=mode,
                             ordering=ordering)
    torch.cuda.synchronize()
    return p, {"G": p.unpack(out["G"]), "U": p.unpack(out["U"]), "V": p.unpack(out["V"]),
               "sigma": p.unpack_sigma(out["sigma"]), "sweeps": out["sweeps"].cpu().numpy()}


def _same(a, b):
    return np.array_equal(np.ascontiguousarray(a).view(np.uint8),
                          np.ascontiguousarray(b).view(np.uint8))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("mode", MODES)
def test_fixed_sweeps_bitwise_vs_oracle(orc, dtype, mode):
    rng = np.random.default_rng(21)
    ns = [2, 4, 6, 10, 16, 32, 34, 64, 66, 8, 2, 40]
    mats = _mats(rng, ns, dtype)
    p, got = _run(mats, dtype, mode, max_sweeps=2, tolf=-1.0)
    assert list(got["sweeps"]) == [-2] * len(ns)
    for k, G0 in enumerate(mats):
        G, U, V, st, swp = orc.kog_sweep(G0, max_sweeps=2, tol_factor=-1.0)
        assert (st, swp) == (1, 2)
        assert _same(got["G"][k], G), (mode, k, ns[k], "G")
        assert _same(got["U"][k], U), (mode, k, ns[k], "U")
        assert _same(got["V"][k], V), (mode, k, ns[k], "V")
        assert _same(got["sigma"][k], np.diag(G)), (mode, k, "sigma")


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("mode", MODES)
def test_larger_orders_bitwise_vs_oracle(orc, dtype, mode):
    """Orders whose U/V update spans several row tiles and several pivots per lane
    (n/2 not a multiple of 64, n/2 > 128, n/2 > 256), one full sweep plus the first
    chunk of the next."""
    ns = [130, 150, 300, 520]
    mats = _mats(np.random.default_rng(31), ns, dtype)
    key = np.dtype(dtype).name
    if key not in _LARGE_REF:  # the oracle's result, shared by the three modes
        _LARGE_REF[key] = [orc.kog_sweep(G0, max_sweeps=2, tol_factor=-1.0) for G0 in mats]
    p, got = _run(mats, dtype, mode, max_sweeps=2, tolf=-1.0)
    assert list(got["sweeps"]) == [-2] * len(ns)
    for k in range(len(ns)):
        G, U, V, st, swp = _LARGE_REF[key][k]
        assert _same(got["G"][k], G), (mode, ns[k], "G")
        assert _same(got["U"][k], U), (mode, ns[k], "U")
        assert _same(got["V"][k], V), (mode, ns[k], "V")


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_converged_modes_identical_and_accurate(orc, dtype):
    rng = np.random.default_rng(5)
    ns = list(2 * rng.integers(8, 65, 24))
    mats = [np.asfortranarray((rng.standard_normal((n, n)) *
                               np.exp2(rng.integers(-30, 31, (n, n)))).astype(dtype)) for n in ns]
    res = {m: _run(mats, dtype, m, max_sweeps=40, tolf=1.0)[1] for m in MODES}
    for m in ("persistent", "graph"):
        assert np.array_equal(res[m]["sweeps"], res["plain"]["sweeps"])
        for k in range(len(ns)):
            for key in ("G", "U", "V"):
                assert _same(res[m][key][k], res["plain"][key][k]), (m, k, key)
    r = res["persistent"]
    eps = 2.0 ** (-53 if dtype == np.float64 else -24)
    assert np.all(r["sweeps"] > 0), r["sweeps"]
    for k, G0 in enumerate(mats):
        n = ns[k]
        G0d = G0.astype(np.float64)
        fro = np.linalg.norm(G0d)
        G = r["G"][k].astype(np.float64)
        assert np.linalg.norm(G - np.diag(np.diag(G))) <= n * eps * fro * (1 + 1e-9)
        sig = np.sort(np.abs(np.diag(G)))[::-1]
        ref = np.linalg.svd(G0d, compute_uv=False)
        assert np.max(np.abs(sig - ref)) <= 50 * n * eps * ref[0]
        U, V = r["U"][k].astype(np.float64), r["V"][k].astype(np.float64)
        assert np.linalg.norm(U.T @ U - np.eye(n)) <= 50 * n * eps
        assert np.linalg.norm(V.T @ V - np.eye(n)) <= 50 * n * eps
        assert np.linalg.norm(U @ np.diag(np.diag(G)) @ V.T - G0d) <= 50 * n * eps * fro
        # the oracle converges after the same number of sweeps (or one off at the boundary)
        if k < 6:
            _, _, _, st, swp = orc.kog_sweep(G0, max_sweeps=40, tol_factor=1.0)
            assert st == 0 and abs(swp - int(r["sweeps"][k])) <= 1


def _off_ratio(G, G0, eps):
    """||offdiag(G)||_F^2 / (n eps ||G0||_F)^2, each sum correctly rounded (math.fsum of
    the binary64 squares: relative error a few 2^-53)."""
    import math

    n = G.shape[0]
    Gd = np.asarray(G, np.float64)
    off = Gd[~np.eye(n, dtype=bool)]
    num = math.fsum((off * off).tolist())
    g0 = np.asarray(G0, np.float64).ravel()
    den = math.fsum((g0 * g0).tolist()) * (n * eps) ** 2
    return num / den


def _check_stop(orc, G0, s_gpu, eps):
    """The stopping decision (Sect. 1: stop once ||offdiag(G)||_F <= n eps ||G_0||_F after
    a sweep) of the device, taken after s_gpu sweeps, against the exact test on the
    oracle's iterates, and against the oracle's own count with its test on.  Any
    binary64 sum of N terms is within (N - 1) 2^-53 (relatively) of the exact one, so a
    decision may differ between the two reductions only when the exact ratio lies
    within delta = (n^2 + 8) 2^-52 of 1; elsewhere both counts must be the same."""
    n = G0.shape[0]
    delta = (n * n + 8) * 2.0 ** -52
    Gp, Up, Vp, _, _ = orc.kog_sweep(G0, max_sweeps=s_gpu - 1, tol_factor=-1.0)
    Gs, _, _, _, _ = orc.kog_sweep(Gp, max_sweeps=1, tol_factor=-1.0, U=Up, V=Vp)
    r_prev = _off_ratio(Gp, G0, eps) if s_gpu > 1 else np.inf
    r_last = _off_ratio(Gs, G0, eps)
    assert r_last <= 1 + delta, (n, s_gpu, r_last)
    assert r_prev > 1 - delta, (n, s_gpu, r_prev)
    _, _, _, st, s_orc = orc.kog_sweep(G0, max_sweeps=s_gpu + 2, tol_factor=1.0)
    assert st == 0
    if s_orc != s_gpu:
        assert abs(s_orc - s_gpu) == 1, (n, s_orc, s_gpu)
        r_dec = r_prev if s_orc > s_gpu else r_last
        assert abs(r_dec - 1) <= delta, (n, s_orc, s_gpu, r_dec)


def test_uniform_workload_full_size_sampled(orc):
    """256 matrices of order 256 (FP64), persistent mode as benchmarked."""
    import torch

    from paper_2407_13116_amd import sweep as sw

    mats = inputs.sweep_uniform()
    p = sw.Packed(mats)
    out = sw.kog_sweep_batch(p, max_sweeps=30, tol_factor=1.0, mode="persistent")
    torch.cuda.synchronize()
    sweeps = out["sweeps"].cpu().numpy()
    assert np.all(sweeps > 0), sweeps
    Gs, Us, Vs = p.unpack(out["G"]), p.unpack(out["U"]), p.unpack(out["V"])
    for k in (0, 137):
        G, U, V, st, swp = orc.kog_sweep(mats[k], max_sweeps=int(sweeps[k]), tol_factor=-1.0)
        assert _same(Gs[k], G) and _same(Us[k], U) and _same(Vs[k], V), k
        ref = np.linalg.svd(mats[k], compute_uv=False)
        sig = np.sort(np.abs(np.diag(G)))[::-1]
        n = mats[k].shape[0]
        # LAPACK's singular values are accurate to n eps sigma_max (absolute) only
        assert np.max(np.abs(sig - ref)) <= 10 * n * 2.0 ** -53 * ref[0]
        _check_stop(orc, mats[k], int(sweeps[k]), 2.0 ** -53)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_uneven_workload_full_size_sampled(orc, dtype):
    """1,000 matrices of uneven order 16..512, persistent mode as benchmarked; three sampled
    matrices (the smallest, a middle and a large order) recomputed by the oracle with the
    same number of sweeps, bit for bit."""
    import torch

    from paper_2407_13116_amd import sweep as sw

    mats = inputs.sweep_uneven(dtype=dtype)
    p = sw.Packed(mats, dtype=dtype)
    out = sw.kog_sweep_batch(p, max_sweeps=60, tol_factor=1.0, mode="persistent")
    torch.cuda.synchronize()
    sweeps = out["sweeps"].cpu().numpy()
    assert np.all(sweeps > 0), sweeps
    Gs, Us, Vs = p.unpack(out["G"]), p.unpack(out["U"]), p.unpack(out["V"])
    ns = np.array([m.shape[0] for m in mats])
    order = np.argsort(ns, kind="stable")
    picks = [int(order[0]), int(order[len(order) // 2]), int(order[int(0.7 * len(order))])]
    for k in picks:
        G, U, V, st, swp = orc.kog_sweep(mats[k], max_sweeps=int(sweeps[k]), tol_factor=-1.0)
        assert _same(Gs[k], G) and _same(Us[k], U) and _same(Vs[k], V), (k, ns[k])
        _check_stop(orc, mats[k], int(sweeps[k]), 2.0 ** (-53 if dtype == np.float64 else -24))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_sigma_gradient(dtype):
    import torch

    from paper_2407_13116_amd import sweep as sw

    rng = np.random.default_rng(9)
    ns = [4, 16, 34, 70]
    mats = _mats(rng, ns, dtype)
    p = sw.Packed(mats, dtype=dtype)
    out = sw.kog_sweep_batch(p, max_sweeps=40, tol_factor=1.0, mode="persistent")
    ds = torch.from_numpy(rng.standard_normal(int(p.n.sum())).astype(dtype)).cuda()
    dG = sw.sigma_grad(p, out["U"], out["V"], ds)
    torch.cuda.synchronize()
    Us, Vs, dGs = p.unpack(out["U"]), p.unpack(out["V"]), p.unpack(dG)
    dsn = p.unpack_sigma(ds)
    eps = 2.0 ** (-53 if dtype == np.float64 else -24)
    for k, n in enumerate(ns):
        want = Us[k].astype(np.float64) @ np.diag(dsn[k].astype(np.float64)) @ Vs[k].astype(np.float64).T
        assert np.max(np.abs(dGs[k] - want)) <= 4 * n * eps * np.max(np.abs(dsn[k])) * 4


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_sigma_gradient_tiles_and_schedule(dtype):
    """The contraction U diag(dsigma) V^T itself, on general (not orthogonal) U and V:
    orders from 1 to 300 (odd ones too, ragged 128 x 128 workgroup tiles and 64 x 64 wave
    tiles, k not a multiple of 4), more matrices than XCDs and in no order of size, so the
    host's largest-first schedule deals several matrices to one XCD.  Every element
    against float64 numpy within the dot product's rounding bound: n + 1 roundings
    (the products u_ik dsigma_k, then the sum) of the absolute terms."""
    import torch

    from paper_2407_13116_amd import sweep as sw

    rng = np.random.default_rng(31)
    ns = [1, 3, 5, 17, 64, 127, 128, 129, 200, 257, 300, 2, 66, 131, 4, 255, 96, 33]
    Um = [np.asfortranarray(rng.standard_normal((n, n)).astype(dtype)) for n in ns]
    Vm = [np.asfortranarray(rng.standard_normal((n, n)).astype(dtype)) for n in ns]
    pu, pv = sw.Packed(Um, dtype=dtype), sw.Packed(Vm, dtype=dtype)
    ds_h = rng.standard_normal(int(pu.n.sum())).astype(dtype)
    dG = sw.sigma_grad(pu, pu.G, pv.G, torch.from_numpy(ds_h).cuda())
    torch.cuda.synchronize()
    got = pu.unpack(dG)
    dsn = pu.unpack_sigma(torch.from_numpy(ds_h))
    eps = 2.0 ** (-53 if dtype == np.float64 else -24)
    for k, n in enumerate(ns):
        U64, V64, d64 = Um[k].astype(np.float64), Vm[k].astype(np.float64), dsn[k].astype(np.float64)
        want = (U64 * d64) @ V64.T
        bound = (n + 1) * eps * (np.abs(U64 * d64) @ np.abs(V64).T) * 1.01 + 1e-300
        assert np.all(np.abs(got[k].astype(np.float64) - want) <= bound), n


def test_sigma_gradient_fd():
    """d sigma_i / dG = u_i v_i^T (sigma sorted, distinct) vs central differences."""
    import torch

    from paper_2407_13116_amd import sweep as sw

    rng = np.random.default_rng(13)
    n = 12
    G0 = np.asfortranarray(rng.standard_normal((n, n)))
    p = sw.Packed([G0])
    out = sw.kog_sweep_batch(p, max_sweeps=40, tol_factor=1.0, mode="persistent")
    sig = p.unpack_sigma(out["sigma"])[0]
    order = np.argsort(-np.abs(sig))
    w = rng.standard_normal(n)
    ds = np.zeros(n)
    ds[order] = w                      # weight w_r on the r-th largest sigma
    dG = sw.sigma_grad(p, out["U"], out["V"], torch.from_numpy(ds).cuda())
    torch.cuda.synchronize()
    got = p.unpack(dG)[0]

    def f(G):
        q = sw.Packed([G])
        o = sw.kog_sweep_batch(q, max_sweeps=40, tol_factor=1.0, mode="persistent")
        s = np.sort(np.abs(q.unpack_sigma(o["sigma"])[0]))[::-1]
        return float(np.dot(w, s))

    h = 1e-6
    fd = np.zeros((n, n))
    for r in range(n):
        for c in range(n):
            Gp, Gm = G0.copy(order="F"), G0.copy(order="F")
            Gp[r, c] += h
            Gm[r, c] -= h
            fd[r, c] = (f(Gp) - f(Gm)) / (2 * h)
    assert np.max(np.abs(got - fd)) <= 1e-6 * np.max(np.abs(fd)) * 10


@pytest.mark.parametrize("mode", MODES)
def test_resume_and_edges(orc, mode):
    import torch

    from paper_2407_13116_amd import sweep as sw

    rng = np.random.default_rng(2)
    mats = _mats(rng, [10, 2, 6], np.float64) + [np.asfortranarray(np.diag([3.0, -1.0, 2.0, 0.5])),
                                                 np.zeros((4, 4), order="F")]
    # 1 + 1 sweeps (resume with the returned U, V) == 2 sweeps, bitwise
    p1 = sw.Packed(mats)
    o1 = sw.kog_sweep_batch(p1, max_sweeps=1, tol_factor=-1.0, mode=mode)
    o1 = sw.kog_sweep_batch(p1, max_sweeps=1, tol_factor=-1.0, mode=mode, U=o1["U"], V=o1["V"])
    p2 = sw.Packed(mats)
    o2 = sw.kog_sweep_batch(p2, max_sweeps=2, tol_factor=-1.0, mode=mode)
    torch.cuda.synchronize()
    for key in ("G", "U", "V"):
        assert torch.equal(o1[key], o2[key]), key
    # diagonal and zero matrices converge after one sweep; order 2 after one
    p3 = sw.Packed(mats)
    o3 = sw.kog_sweep_batch(p3, max_sweeps=10, tol_factor=1.0, mode=mode)
    sweeps = o3["sweeps"].cpu().numpy()
    assert sweeps[1] == 1 and sweeps[3] == 1 and sweeps[4] == 1, sweeps
    sig = p3.unpack_sigma(o3["sigma"])
    assert sorted(sig[3]) == [0.5, 1.0, 2.0, 3.0]
    assert np.all(sig[4] == 0)


def test_persistent_order_limit_names_mode0():
    """Orders whose step parameters do not fit a workgroup's LDS are refused by the
    persistent modes with a message naming mode 0 (nothing is launched)."""
    from paper_2407_13116_amd import KSVD2Error
    from paper_2407_13116_amd import sweep as sw

    n = 3400
    p = sw.Packed([np.asfortranarray(np.eye(n))])
    with pytest.raises(KSVD2Error, match="mode 0"):
        sw.kog_sweep_batch(p, max_sweeps=1, tol_factor=-1.0, mode="persistent")


def test_mode0_largest_order_one_sweep():
    """Order 8192 (the largest accepted; one row of its U/V tile exceeds 64 KB of LDS in
    binary64): one plain-mode sweep keeps U, V orthogonal and U^T G0 V equal to the
    iterated G, both to a few n eps, and lowers the off-diagonal norm (checked on the
    device)."""
    import torch

    from paper_2407_13116_amd import sweep as sw

    n = 8192
    g = torch.Generator(device="cuda").manual_seed(8192)
    G0 = torch.randn((n, n), dtype=torch.float64, device="cuda", generator=g)
    p = sw.Packed.__new__(sw.Packed)
    p.n = np.array([n], dtype=np.int32)
    p.off = np.array([0], dtype=np.int64)
    p.soff = np.array([0], dtype=np.int64)
    p.G = G0.t().contiguous().reshape(-1).clone()   # column-major G0
    p.dtype = p.G.dtype
    out = sw.kog_sweep_batch(p, max_sweeps=1, tol_factor=-1.0, mode="plain")
    torch.cuda.synchronize()
    assert int(out["sweeps"][0]) == -1
    U = out["U"].reshape(n, n).t()                  # column-major -> matrix view
    V = out["V"].reshape(n, n).t()
    G = out["G"].reshape(n, n).t()
    eps = 2.0 ** -53
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    assert float(torch.linalg.norm(U.t().contiguous() @ U.contiguous() - eye)) <= 10 * n * eps
    assert float(torch.linalg.norm(V.t().contiguous() @ V.contiguous() - eye)) <= 10 * n * eps
    R = U.t().contiguous() @ G0 @ V.contiguous()
    assert float(torch.linalg.norm(R - G)) <= 10 * n * eps * float(torch.linalg.norm(G0))
    # one sweep of a large Gaussian matrix lowers the off-diagonal norm (to about
    # 0.76 of it here; the first sweeps of the two-sided method move slowly)
    off0 = float(torch.linalg.norm(G0 - torch.diag(torch.diagonal(G0))))
    off = float(torch.linalg.norm(G - torch.diag(torch.diagonal(G))))
    assert off < 0.9 * off0


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("mode", MODES)
def test_sorted_convention(dtype, mode):
    """sort=True: sigma descending (ties in index order), U and V columns permuted the
    same way -- bit for bit the unsorted result permuted by a stable sort -- and
    G0 = U diag(sigma) V^T."""
    import torch

    rng = np.random.default_rng(41)
    ns = [2, 6, 34, 66, 130, 300]
    mats = _mats(rng, ns, dtype)
    mats.append(np.asfortranarray(np.diag([1.0, 3.0, 3.0, 2.0, 0.0, 3.0]).astype(dtype)))
    ns.append(6)
    _, ref = _run(mats, dtype, mode, max_sweeps=40, tolf=1.0)
    from paper_2407_13116_amd import sweep as sw

    p = sw.Packed(mats, dtype=dtype)
    out = sw.kog_sweep_batch(p, max_sweeps=40, tol_factor=1.0, mode=mode, sort=True)
    torch.cuda.synchronize()
    sig, Us, Vs = p.unpack_sigma(out["sigma"]), p.unpack(out["U"]), p.unpack(out["V"])
    eps = 2.0 ** (-53 if dtype == np.float64 else -24)
    for k, G0 in enumerate(mats):
        s0 = ref["sigma"][k]
        perm = np.argsort(-s0, kind="stable")
        assert _same(sig[k], s0[perm]), k
        assert np.all(np.diff(sig[k].astype(np.float64)) <= 0), k
        assert _same(Us[k], ref["U"][k][:, perm]) and _same(Vs[k], ref["V"][k][:, perm]), k
        R = Us[k].astype(np.float64) @ np.diag(sig[k].astype(np.float64)) @ Vs[k].astype(np.float64).T
        assert np.linalg.norm(R - G0) <= 50 * ns[k] * eps * max(np.linalg.norm(G0), 1e-300)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("mode", MODES)
def test_global_scaling_bitwise_vs_oracle(orc, dtype, mode):
    """Matrices whose largest entries sit a few binades below the overflow threshold
    (scaled by 2^s_G < 1 before the sweep and back after it), mixed with ordinary ones:
    G, U, V bit for bit equal to the oracle after two fixed sweeps, all finite."""
    e_nu = 1023 if np.dtype(dtype) == np.float64 else 127
    rng = np.random.default_rng(77)
    ns = [8, 34, 66, 130]
    mats = _mats(rng, ns, dtype)
    for k in (0, 2):
        mats[k] = np.asfortranarray((mats[k].astype(np.float64) * 2.0 ** (e_nu - 6)).astype(dtype))
    p, got = _run(mats, dtype, mode, max_sweeps=2, tolf=-1.0)
    for k, G0 in enumerate(mats):
        G, U, V, st, swp = orc.kog_sweep(G0, max_sweeps=2, tol_factor=-1.0)
        assert np.all(np.isfinite(got["G"][k])), (mode, ns[k])
        assert _same(got["G"][k], G), (mode, ns[k], "G")
        assert _same(got["U"][k], U), (mode, ns[k], "U")
        assert _same(got["V"][k], V), (mode, ns[k], "V")


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("mode", MODES)
def test_round_robin_ordering_bitwise_vs_oracle(orc, dtype, mode):
    rng = np.random.default_rng(24)
    ns = [2, 4, 6, 10, 16, 34, 66, 8, 130, 260]
    mats = _mats(rng, ns, dtype)
    p, got = _run(mats, dtype, mode, max_sweeps=2, tolf=-1.0, ordering="round-robin")
    assert list(got["sweeps"]) == [-2] * len(ns)
    for k, G0 in enumerate(mats):
        G, U, V, st, swp = orc.kog_sweep(G0, max_sweeps=2, tol_factor=-1.0, ordering=0)
        assert (st, swp) == (1, 2)
        assert _same(got["G"][k], G), (mode, k, ns[k], "G")
        assert _same(got["U"][k], U), (mode, k, ns[k], "U")
        assert _same(got["V"][k], V), (mode, k, ns[k], "V")


@pytest.mark.parametrize("ordering", ["round-robin", "modulus"])
def test_orderings_converge_to_lapack(ordering):
    rng = np.random.default_rng(25)
    ns = [4, 16, 64, 128]
    mats = _mats(rng, ns, np.float64)
    p, got = _run(mats, np.float64, "persistent", max_sweeps=40, tolf=1.0, ordering=ordering)
    assert np.all(got["sweeps"] > 0)
    for k, G0 in enumerate(mats):
        ref = np.linalg.svd(G0, compute_uv=False)
        sig = np.sort(np.abs(got["sigma"][k]))[::-1]
        assert np.max(np.abs(sig - ref)) <= 40 * ns[k] * 2.0 ** -53 * ref[0]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("mode", MODES)
def test_sparse_and_structured_bitwise(orc, dtype, mode):
    """Matrices with many exact zeros (every zero pattern of the 2x2 pivots occurs),
    rank-one and rank-deficient ones, wide exponent ranges, and signed zeros: two sweeps
    bit for bit against the oracle."""
    rng = np.random.default_rng(31)
    mats = []
    for n in (8, 16, 30, 64):
        A = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.3)
        mats.append(A)
        u, v = rng.standard_normal(n), rng.standard_normal(n)
        mats.append(np.outer(u, v))
        B = rng.standard_normal((n, n))
        B[:, n // 2:] = B[:, : n - n // 2] * 2.0          # rank n/2 exactly
        mats.append(B)
        C = rng.standard_normal((n, n)) * np.exp2(rng.integers(-60, 61, (n, n)))
        mats.append(C)
        D = np.where(rng.random((n, n)) < 0.5, -0.0, 0.0)
        D[np.arange(n), np.arange(n)] = rng.standard_normal(n)
        mats.append(D)
    mats = [np.asfortranarray(m.astype(dtype)) for m in mats]
    p, got = _run(mats, dtype, mode, max_sweeps=2, tolf=-1.0)
    for k, G0 in enumerate(mats):
        G, U, V, st, swp = orc.kog_sweep(G0, max_sweeps=2, tol_factor=-1.0)
        assert _same(got["G"][k], G), (mode, k, "G")
        assert _same(got["U"][k], U), (mode, k, "U")
        assert _same(got["V"][k], V), (mode, k, "V")



@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_two_step_passes_every_block_size(orc, dtype):
    """The persistent kernel at every workgroup size (in place for orders up to 256
    in workgroups of up to 512 lanes, through the second buffer otherwise, paired U/V
    rotations or not): orders at the boundaries of the lane layouts (n/2 = 2, 3, 63,
    64, 65, 128, 129, 192, 193, 256), bit for bit against the oracle over a sweep and
    a half."""
    import torch

    from paper_2407_13116_amd import sweep as sw

    tdt = torch.float64 if dtype == np.float64 else torch.float32
    ns = [4, 6, 126, 128, 130, 256, 258, 202, 384, 386, 512]
    mats = _mats(np.random.default_rng(44), ns, dtype)
    ref = [orc.kog_sweep(G0, max_sweeps=2, tol_factor=-1.0) for G0 in mats]
    try:
        for block in (256, 512, 1024):
            for bucket in range(5):
                sw.set_tuning(tdt, bucket, block)
            p, got = _run(mats, dtype, "persistent", max_sweeps=2, tolf=-1.0)
            for k in range(len(ns)):
                G, U, V, st, swp = ref[k]
                assert _same(got["G"][k], G), (block, ns[k], "G")
                assert _same(got["U"][k], U), (block, ns[k], "U")
                assert _same(got["V"][k], V), (block, ns[k], "V")
    finally:
        sw.reset_tuning()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_every_tuning_knob_bitwise(orc, dtype):
    """The schedule knobs the autotuner searches (steps per U/V update, two steps of G
    per pass, the in-place pass, a cap on U/V tile rows, with every workgroup size)
    change no bit: one and a half sweeps of orders across the buckets against the
    oracle, under each setting, both orderings."""
    import torch

    from paper_2407_13116_amd import sweep as sw

    tdt = torch.float64 if dtype == np.float64 else torch.float32
    ns = [6, 64, 66, 130, 256, 258, 300]
    mats = _mats(np.random.default_rng(45), ns, dtype)
    settings = [dict(chunk=2), dict(chunk=16, rows=8), dict(two=0), dict(inplace=0, block=512),
                dict(chunk=32, two=0, rows=1, block=1024), dict(inplace=0, chunk=64, rows=24),
                dict(block=256, chunk=8)]
    try:
        for ordering in ("modulus", "round-robin"):
            ref = [orc.kog_sweep(G0, max_sweeps=2, tol_factor=-1.0,
                                 ordering=1 if ordering == "modulus" else 0) for G0 in mats]
            for st in settings:
                sw.reset_tuning()
                sw.set_tuning(tdt, -1, **st)
                p, got = _run(mats, dtype, "persistent", max_sweeps=2, tolf=-1.0,
                              ordering=ordering)
                for k in range(len(ns)):
                    G, U, V, _, _ = ref[k]
                    for key, want in (("G", G), ("U", U), ("V", V)):
                        assert _same(got[key][k], want), (ordering, st, ns[k], key)
    finally:
        sw.reset_tuning()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("mode", MODES)
def test_dynamic_ordering_bitwise_vs_oracle(orc, dtype, mode):
    """The dynamic ordering (a greedy matching of every step's weights): two sweeps
    bit for bit against the oracle in every mode, on orders 2 .. 258 and on sparse and
    integer matrices whose weights tie (zeros, repeated magnitudes), where the index
    order of equal weights decides; then converged runs with the oracle's sweep count."""
    rng = np.random.default_rng(91)
    ns = [2, 4, 6, 10, 16, 34, 64, 66, 130]
    mats = _mats(rng, ns, dtype)
    for n in (8, 40, 258):
        A = rng.choice([0.0, 1.0, -1.0, 2.0], (n, n)) * (rng.random((n, n)) < 0.3)
        mats.append(np.asfortranarray(A.astype(dtype)))
    ns = [m.shape[0] for m in mats]
    p, got = _run(mats, dtype, mode, max_sweeps=2, tolf=-1.0, ordering="dynamic")
    for k, G0 in enumerate(mats):
        G, U, V, _, _ = orc.kog_sweep(G0, max_sweeps=2, tol_factor=-1.0, ordering=2)
        assert _same(got["G"][k], G), (mode, ns[k], "G")
        assert _same(got["U"][k], U), (mode, ns[k], "U")
        assert _same(got["V"][k], V), (mode, ns[k], "V")
    small = mats[:7]
    p, got = _run(small, dtype, mode, max_sweeps=30, tolf=1.0, ordering="dynamic")
    for k, G0 in enumerate(small):
        G, U, V, st, swp = orc.kog_sweep(G0, max_sweeps=30, tol_factor=1.0, ordering=2)
        assert st == 0 and int(got["sweeps"][k]) == swp, (mode, ns[k])
        assert _same(got["G"][k], G) and _same(got["U"][k], U), (mode, ns[k])


def test_autotuner_installs_a_valid_schedule(tmp_path, monkeypatch):
    """The autotuner's coordinate search on a small uneven batch: one setting per bucket
    present, each within the knobs' ranges and installed in the library's table; a
    second call reuses the cache without timing."""
    import torch

    from paper_2407_13116_amd import autotune
    from paper_2407_13116_amd import sweep as sw

    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    mats = _mats(np.random.default_rng(46), [20, 40, 100, 130, 200, 300], np.float64)
    try:
        chosen = autotune.tune(mats, torch.float64, sample=4, force=True)
        assert sorted(chosen) == [0, 1, 2, 3]
        for b, st in chosen.items():
            assert st["block"] in (256, 512, 1024) and st["two"] in (0, 1)
            assert st["inplace"] in (0, 1) and st["chunk"] in (16, 32, 64, 128)
            assert st["rows"] in (0, 16, 32, 64)
            assert sw.get_tuning(torch.float64, b) == st
        sw.reset_tuning()
        again = autotune.tune(mats, torch.float64, sample=4)
        assert again == chosen
    finally:
        sw.reset_tuning()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_large_orders_persistent_matches_plain(dtype):
    """Orders whose two steps' parameters do not fit the LDS beside 16 U/V tile rows
    (the second step's come from the step table): one sweep in the persistent mode and
    in mode 0 (per-step launches, one step per pass), bit for bit."""
    ns = [1024, 2000]
    mats = _mats(np.random.default_rng(61), ns, dtype)
    _, a = _run(mats, dtype, "persistent", max_sweeps=1, tolf=-1.0)
    _, b = _run(mats, dtype, "plain", max_sweeps=1, tolf=-1.0)
    for k in range(len(ns)):
        for key in ("G", "U", "V"):
            assert _same(a[key][k], b[key][k]), (ns[k], key)


def test_graph_replays_match_eager():
    """Mode 2 captures the persistent launches once per argument set and replays the
    graph: the same buffers, G re-filled by eager copies between the replays (with other
    eager work and synchronizations in between); every replay bit for bit equal to mode 1
    on its own buffers."""
    import ctypes

    import torch

    from paper_2407_13116_amd import _lib
    from paper_2407_13116_amd import sweep as sw

    mats = _mats(np.random.default_rng(77), [64, 130, 256, 6], np.float64)
    p = sw.Packed(mats, dtype=np.float64)
    G0 = p.G.clone()
    ref = sw.kog_sweep_batch(sw.Packed(mats, dtype=np.float64), max_sweeps=3, tol_factor=1.0,
                             mode="persistent")
    torch.cuda.synchronize()
    L = _lib.lib()
    n = np.ascontiguousarray(p.n)
    off = np.ascontiguousarray(p.off)
    U, V = torch.empty_like(p.G), torch.empty_like(p.G)
    sigma = torch.empty(int(n.sum()), dtype=p.G.dtype, device="cuda")
    sweeps = torch.empty(len(n), dtype=torch.int32, device="cuda")
    need = sw.workspace_bytes(p.G.dtype, n)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    st = torch.cuda.Stream()
    for rep in range(3):
        with torch.cuda.stream(st):
            p.G.copy_(G0)
            junk = torch.randn(1 << 20, device="cuda").sum()  # other eager work
            rc = L.kog_sweep_batch(1, len(n), n.ctypes.data_as(ctypes.c_void_p),
                                   off.ctypes.data_as(ctypes.c_void_p), p.G.data_ptr(),
                                   U.data_ptr(), V.data_ptr(), sigma.data_ptr(),
                                   sweeps.data_ptr(), 3, 1.0, 0, 2, 1, ws.data_ptr(), need,
                                   ctypes.c_void_p(st.cuda_stream))
        assert rc == 0, _lib.lib().ksvd2_last_error()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for key, got in (("G", p.G), ("U", U), ("V", V), ("sigma", sigma), ("sweeps", sweeps)):
            a = got.cpu().numpy()
            b = ref[key].cpu().numpy()
            assert _same(a, b), (rep, key)
