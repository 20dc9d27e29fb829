"""GPU parity of the adjoint (and of the autograd path built on it).

* forward in the autograd layout: bitwise equal to the oracle (U, V, plain S);
* backward kernel vs the oracle's float64 formula on the same (U, S, V): agreement to a
  bound derived from the arithmetic, 16 eps (|dS1| + |dS2| + (|dU| + |dV|)(1/|s1-s2| +
  1/(s1+s2))), where eps is the working precision's unit roundoff;
* the 4,096-matrix finite-difference subset of the differentiable workload, through
  torch.autograd: general matrices (full loss, FP64 vs FP64 differences to 1e-6; a
  gauge-invariant loss for FP32 vs FP64 differences to 1e-3), near-degenerate matrices
  (the polar-factor loss, differences through a 300-bit SVD; FP32 uses tau = 2^-12),
  rank-deficient matrices (first singular triple);
* not checked by finite differences: general upstream dU and dV on the near-degenerate
  subset in FP32, and sigma_1 and sigma_2 weighted differently there.  With sigma1/sigma2 -
  1 < 1e-6 the singular vectors, and any loss that tells the two triples apart, change by
  eps/(sigma1 - sigma2) ~ 6% under binary32 rounding, so no finite difference resolves
  them to 1e-3; the adjoint's arithmetic on those matrices is still checked against the
  oracle adjoint within the derived bound (test_backward_kernel_vs_oracle);
* the full 2^22 batch in both precisions: finite, and sampled outputs vs the oracle;
* the kernels' 16-byte vector paths and their element-wise paths give the same bits.
"""
import numpy as np
import pytest

from gpu_util import to_dev
from paper_2407_13116_amd import inputs

pytestmark = pytest.mark.gpu


def _eps(dtype):
    return 2.0 ** (-53 if np.dtype(dtype) == np.float64 else -24)


def _gpu_fwd(G):
    import torch

    from paper_2407_13116_amd import api

    U, S, V = api.svd2x2_raw(to_dev(G)[0])
    torch.cuda.synchronize()
    return U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()


def _bound(U, S, V, dS, dU, dV, dtype):
    s1, s2 = S[:, 0].astype(np.float64), S[:, 1].astype(np.float64)
    with np.errstate(divide="ignore"):
        idm = np.where(s1 != s2, 1 / np.abs(s1 - s2), 0.0)
        ism = np.where(s1 + s2 != 0, 1 / (s1 + s2), 0.0)
    g = np.abs(dU).reshape(len(U), -1).sum(1) + np.abs(dV).reshape(len(U), -1).sum(1)
    return 16 * _eps(dtype) * (np.abs(dS).sum(1) + g * (idm + ism))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_backward_kernel_vs_oracle(orc, dtype):
    import torch

    from paper_2407_13116_amd import api

    G, dS, dU, dV, lab = inputs.diff_batch(dtype, B=1 << 16)
    # forward: bitwise against the oracle
    U, S, V = _gpu_fwd(G)
    o = orc.ksvd2(*inputs.soa_from_mats(G))
    Uo, Vo = orc.full_uv(o)
    assert np.array_equal(U.astype(np.float64), Uo) and np.array_equal(V.astype(np.float64), Vo)
    assert np.array_equal(S[:, 0], o["s1"]) and np.array_equal(S[:, 1], o["s2"])
    # backward on the GPU's own (U, S, V)
    t = to_dev(U, S, V, dS, dU, dV)
    dG = api.svd2x2_backward(*t).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    want = orc.svd2_backward(U, S, V, dS, dU, dV)
    err = np.abs(dG - want).reshape(len(G), -1).max(1)
    bound = _bound(U, S, V, dS, dU, dV, dtype)
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, (bad[:5], err[bad[:5]], bound[bad[:5]], lab[bad[:5]])
    # optional inputs: null dU/dV == zeros
    dG2 = api.svd2x2_backward(t[0], t[1], t[2], t[3]).cpu().numpy().astype(np.float64)
    want2 = orc.svd2_backward(U, S, V, dS)
    assert np.all(np.abs(dG2 - want2).reshape(len(G), -1).max(1)
                  <= _bound(U, S, V, dS, 0 * dU, 0 * dV, dtype))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_vector_and_element_paths_agree(dtype):
    """Tensors on 16-byte boundaries take the kernels' vector loads and stores; a view
    one element off such a boundary takes the element-wise path: same bits."""
    import torch

    from paper_2407_13116_amd import api

    G, dS, dU, dV, _ = inputs.diff_batch(dtype, B=1 << 12)
    tdt = torch.float64 if np.dtype(dtype) == np.float64 else torch.float32

    def shifted(x):
        x = torch.as_tensor(x).to("cuda")
        flat = torch.empty(x.numel() + 1, dtype=tdt, device="cuda")
        v = flat[1:].view(x.shape)
        v.copy_(x)
        assert v.data_ptr() % 16 != 0
        return v

    t = to_dev(G, dS, dU, dV)
    U, S, V = api.svd2x2_raw(t[0])
    U2, S2, V2 = api.svd2x2_raw(shifted(G))
    for a, b in ((U, U2), (S, S2), (V, V2)):
        assert torch.equal(a, b)
    dG = api.svd2x2_backward(U, S, V, t[1], t[2], t[3])
    dG2 = api.svd2x2_backward(shifted(U), shifted(S), shifted(V), shifted(t[1]), shifted(t[2]),
                              shifted(t[3]))
    torch.cuda.synchronize()
    assert torch.equal(dG, dG2)


def _fd_gpu(G64, loss, h_rel=1e-6):
    """Central differences of loss(U, S, V) through the GPU forward (float64)."""
    B = G64.shape[0]
    grad = np.zeros_like(G64)
    gmax = np.abs(G64).reshape(B, -1).max(1)
    for r in range(2):
        for c in range(2):
            h = h_rel * np.maximum(np.abs(G64[:, r, c]), 1e-3 * gmax)
            Gp, Gm = G64.copy(), G64.copy()
            Gp[:, r, c] += h
            Gm[:, r, c] -= h
            grad[:, r, c] = (loss(*_gpu_fwd(Gp)) - loss(*_gpu_fwd(Gm))) / (2 * h)
    return grad


def _autograd(G, loss_t, tau=0.0):
    import torch

    from paper_2407_13116_amd import api

    Gt = to_dev(G)[0].requires_grad_(True)
    U, S, V = api.svd2x2(Gt, tau)
    loss_t(U, S, V).sum().backward()
    torch.cuda.synchronize()
    return Gt.grad.cpu().numpy().astype(np.float64)


def _rel(a, b):
    scale = np.maximum(np.abs(b).reshape(len(b), -1).max(1), 1e-300)
    return np.abs(a - b).reshape(len(b), -1).max(1) / scale


def _subset():
    G, dS, dU, dV, lab = inputs.diff_batch(np.float64, B=1 << 22)
    return G[:4096], dS[:4096], dU[:4096], dV[:4096], lab[:4096]


def test_fd_general_f64_full_loss():
    import torch

    G, dS, dU, dV, lab = _subset()
    sel = lab == 0
    G, dS, dU, dV = G[sel], dS[sel], dU[sel], dV[sel]
    td = to_dev(dS, dU, dV)

    def loss_t(U, S, V):
        return (td[0] * S).sum(1) + (td[1] * U).sum((1, 2)) + (td[2] * V).sum((1, 2))

    def loss_n(U, S, V):
        return (dS * S).sum(1) + (dU * U).sum((1, 2)) + (dV * V).sum((1, 2))

    got = _autograd(G, loss_t)
    fd = _fd_gpu(G, loss_n)
    r = _rel(got, fd)
    assert r.max() <= 1e-6, (r.max(), int(np.argmax(r)))
    assert torch.cuda.is_available()


def test_fd_general_f32_invariant_loss():
    G, dS, dU, dV, lab = _subset()
    sel = lab == 0
    G, dS, W, w = G[sel], dS[sel], dU[sel], dV[sel][:, 0, :]
    G32 = G.astype(np.float32)
    td = to_dev(dS.astype(np.float32), W.astype(np.float32), w.astype(np.float32))

    def loss_t(U, S, V):   # dS.S + <W, U diag(w) V^T>: invariant under the sign gauge
        UV = (U[:, :, None, :] * td[2][:, None, None, :] * V[:, None, :, :]).sum(-1)
        return (td[0] * S).sum(1) + (td[1] * UV).sum((1, 2))

    def loss_n(U, S, V):
        UV = np.einsum("bik,bk,bjk->bij", U, w, V)
        return (dS * S).sum(1) + (W * UV).sum((1, 2))

    got = _autograd(G32, loss_t)
    fd = _fd_gpu(G32.astype(np.float64), loss_n)
    r = _rel(got, fd)
    assert r.max() <= 1e-3, (r.max(), int(np.argmax(r)))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_fd_near_degenerate_polar_loss(dtype):
    """sigma1/sigma2 - 1 < 1e-6.  FP64 with the exact formula (tau = 0) to 1e-6; FP32 with
    the broadened 1/(s1-s2) (tau = 2^-12), since FP32 rounding of the skew parts is
    amplified by 1/(s1-s2) there, and with equal weights on sigma1 and sigma2, to 1e-3."""
    from test_oracle_sweep_bwd import _mp_polar_loss_grad

    G, dS, dU, dV, lab = _subset()
    sel = lab == 1
    G, dS, W = G[sel][:96], dS[sel][:96], dU[sel][:96]
    if dtype == np.float32:
        # with sigma1 ~ sigma2 the split of dS.S between the two triples depends on u_i, v_i,
        # which binary32 resolves only to eps/(s1 - s2) ~ 6%: weigh both equally (the trace
        # norm), which is well-conditioned there
        dS = np.repeat(dS.mean(1, keepdims=True), 2, axis=1)
    Gd = G.astype(dtype)
    td = to_dev(dS.astype(dtype), W.astype(dtype))

    def loss_t(U, S, V):
        UV = (U[:, :, None, :] * V[:, None, :, :]).sum(-1)   # U V^T without a batched matmul
        return (td[0] * S).sum(1) + (td[1] * UV).sum((1, 2))

    tau = 0.0 if dtype == np.float64 else 2.0 ** -12
    got = _autograd(Gd, loss_t, tau)
    fd = np.stack([_mp_polar_loss_grad(Gd[i].astype(np.float64), dS[i], W[i])
                   for i in range(len(G))])
    r = _rel(got, fd)
    assert r.max() <= (1e-6 if dtype == np.float64 else 1e-3), r.max()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_fd_rank_deficient_first_triple(dtype):
    G, dS, dU, dV, lab = _subset()
    sel = lab == 2
    G, dS, W = G[sel], dS[sel], dU[sel]
    Gd = G.astype(dtype)
    td = to_dev(dS[:, 0].astype(dtype), W.astype(dtype))

    def loss_t(U, S, V):
        return td[0] * S[:, 0] + (td[1] * U[:, :, 0, None] * V[:, None, :, 0]).sum((1, 2))

    def loss_n(U, S, V):
        return dS[:, 0] * S[:, 0] + np.einsum("bij,bi,bj->b", W, U[:, :, 0], V[:, :, 0])

    got = _autograd(Gd, loss_t)
    assert np.all(np.isfinite(got))
    fd = _fd_gpu(Gd.astype(np.float64), loss_n)
    r = _rel(got, fd)
    assert r.max() <= (1e-6 if dtype == np.float64 else 1e-3), r.max()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_full_batch_fwd_bwd(orc, dtype):
    """The whole 2^22 differentiable batch through forward + backward, as benchmarked."""
    import torch

    from paper_2407_13116_amd import api

    G, dS, dU, dV, lab = inputs.diff_batch(dtype)
    t = to_dev(G, dS, dU, dV)
    U, S, V = api.svd2x2_raw(t[0])
    dG = api.svd2x2_backward(U, S, V, t[1], t[2], t[3])
    torch.cuda.synchronize()
    Un, Sn, Vn, dGn = (x.cpu().numpy() for x in (U, S, V, dG))
    assert np.all(np.isfinite(dGn[lab != 1]))
    rng = np.random.default_rng(3)
    idx = np.unique(rng.integers(0, len(G), 1 << 14))
    want = orc.svd2_backward(Un[idx], Sn[idx], Vn[idx], dS[idx], dU[idx], dV[idx])
    err = np.abs(dGn[idx].astype(np.float64) - want).reshape(len(idx), -1).max(1)
    assert np.all(err <= _bound(Un[idx], Sn[idx], Vn[idx], dS[idx], dU[idx], dV[idx], dtype))


def _planes4(M):
    """[B,2,2] -> [4,B] planes of the entries (1,1), (2,1), (1,2), (2,2)."""
    return np.ascontiguousarray(np.stack([M[:, 0, 0], M[:, 1, 0], M[:, 0, 1], M[:, 1, 1]]))


def _full_from_planes(c, s, info, bit):
    """U = [c -d s; s d c] with d = -1 where the info bit is set."""
    d = np.where(info & bit, -1.0, 1.0).astype(c.dtype)
    return np.stack([np.stack([c, -d * s], -1), np.stack([s, d * c], -1)], 1)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_backward_planes_vs_oracle_and_full_layout(orc, dtype):
    """ksvd2_batch_backward on the SoA forward's own planes (ragged batch): within the
    derived bound of the oracle adjoint, and bit for bit the [B,2,2] adjoint on the
    expanded U, V; null upstream gradients equal zero ones, bit for bit."""
    import torch

    from paper_2407_13116_amd import api

    B = (1 << 16) + 37
    G, dS, dU, dV, lab = inputs.diff_batch(dtype, B=B)
    fwd = api.ksvd2_batch(*to_dev(*inputs.soa_from_mats(G)), plain=True)
    h = {k: v.cpu().numpy() for k, v in fwd.items()}
    U = _full_from_planes(h["cu"], h["su"], h["info"], 1 << 8)
    V = _full_from_planes(h["cv"], h["sv"], h["info"], 1 << 9)
    S = np.stack([h["s1"], h["s2"]], 1)
    o = orc.ksvd2(*inputs.soa_from_mats(G))
    Uo, Vo = orc.full_uv(o)
    assert np.array_equal(U.astype(np.float64), Uo) and np.array_equal(V.astype(np.float64), Vo)
    ds1, ds2, pU, pV = to_dev(dS[:, 0], dS[:, 1], _planes4(dU), _planes4(dV))
    dGp = api.ksvd2_backward_soa(fwd, ds1, ds2, pU, pV)
    torch.cuda.synchronize()
    g = dGp.cpu().numpy()
    dG = np.stack([np.stack([g[0], g[2]], -1), np.stack([g[1], g[3]], -1)], 1)
    want = orc.svd2_backward(U, S, V, dS, dU, dV)
    err = np.abs(dG.astype(np.float64) - want).reshape(B, -1).max(1)
    bound = _bound(U, S, V, dS, dU, dV, dtype)
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, (bad[:5], err[bad[:5]], bound[bad[:5]], lab[bad[:5]])
    # the [B,2,2] kernel on the expanded matrices: the same bits
    t = to_dev(U, S, V, dS, dU, dV)
    dGf = api.svd2x2_backward(*t).cpu().numpy()
    assert np.array_equal(dGf.view(np.uint8), np.ascontiguousarray(dG).view(np.uint8))
    # null upstream gradients
    for args, full in (((None, None, pU, pV), (t[0], t[1], t[2], None, t[4], t[5])),
                       ((ds1, ds2, None, None), (t[0], t[1], t[2], t[3], None, None)),
                       ((None, None, None, pV), (t[0], t[1], t[2], None, None, t[5]))):
        g = api.ksvd2_backward_soa(fwd, *args).cpu().numpy()
        a = np.stack([np.stack([g[0], g[2]], -1), np.stack([g[1], g[3]], -1)], 1)
        b = api.svd2x2_backward(*full).cpu().numpy()
        assert np.array_equal(a.view(np.uint8), np.ascontiguousarray(b).view(np.uint8))


def test_backward_planes_past_one_launch(orc):
    """2^28 + 4,099 FP32 matrices (more than one launch of 2^28): outputs around the
    launch boundary and at both ends within the bound of the oracle adjoint."""
    import torch

    from paper_2407_13116_amd import api

    B = (1 << 28) + 4099
    gen = torch.Generator(device="cuda").manual_seed(11)
    ang = torch.rand(2, B, device="cuda", generator=gen, dtype=torch.float32) * 6.2831855
    info = (torch.randint(0, 4, (B,), device="cuda", generator=gen, dtype=torch.int32) << 8)
    sv = torch.rand(2, B, device="cuda", generator=gen, dtype=torch.float32) + 0.5
    fwd = {"cu": torch.cos(ang[0]), "su": torch.sin(ang[0]), "cv": torch.cos(ang[1]),
           "sv": torch.sin(ang[1]), "info": info,
           "s1": torch.maximum(sv[0], sv[1]).contiguous(), "s2": torch.minimum(sv[0], sv[1]).contiguous()}
    del ang, sv
    ds = torch.randn(2, B, device="cuda", generator=gen, dtype=torch.float32)
    pU = torch.randn(4, B, device="cuda", generator=gen, dtype=torch.float32)
    pV = torch.randn(4, B, device="cuda", generator=gen, dtype=torch.float32)
    out = api.ksvd2_backward_soa(fwd, ds[0], ds[1], pU, pV)
    torch.cuda.synchronize()
    L = 1 << 28
    idx = np.concatenate([np.arange(0, 64), np.arange(L - 300, L + 300), np.arange(B - 64, B)])
    it = torch.from_numpy(idx).cuda()
    h = {k: v[it].cpu().numpy() for k, v in fwd.items()}
    U = _full_from_planes(h["cu"], h["su"], h["info"], 1 << 8)
    V = _full_from_planes(h["cv"], h["sv"], h["info"], 1 << 9)
    S = np.stack([h["s1"], h["s2"]], 1)
    dSn = ds[:, it].cpu().numpy().T.copy()
    p, q = pU[:, it].cpu().numpy(), pV[:, it].cpu().numpy()
    dUn = np.stack([np.stack([p[0], p[2]], -1), np.stack([p[1], p[3]], -1)], 1)
    dVn = np.stack([np.stack([q[0], q[2]], -1), np.stack([q[1], q[3]], -1)], 1)
    g = out[:, it].cpu().numpy()
    dG = np.stack([np.stack([g[0], g[2]], -1), np.stack([g[1], g[3]], -1)], 1)
    want = orc.svd2_backward(U, S, V, dSn, dUn, dVn)
    err = np.abs(dG.astype(np.float64) - want).reshape(len(idx), -1).max(1)
    assert np.all(err <= _bound(U, S, V, dSn, dUn, dVn, np.float32)), err.max()
    del fwd, ds, pU, pV, out
    torch.cuda.empty_cache()
