"""The usage example of README.md runs as written (small sizes) and gives consistent
results: the autograd, SoA and complex entry points and the square and rectangular
sweeps."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_readme_example():
    import torch

    from paper_2407_13116_amd import api, sweep

    G = torch.randn(1 << 12, 2, 2, dtype=torch.float64, device="cuda", requires_grad=True)
    U, S, V = api.svd2x2(G)
    planes = [G.detach()[:, i, j].contiguous() for i, j in ((0, 0), (1, 0), (0, 1), (1, 1))]
    out = api.ksvd2_batch(*planes)
    assert torch.equal(out["s1"], S[:, 0].detach()) and torch.equal(out["s2"], S[:, 1].detach())
    S.sum().backward()
    assert torch.isfinite(G.grad).all()
    Gc = torch.randn(64, 2, 2, dtype=torch.complex128, device="cuda")
    Uc, Sc, Vc = api.ksvd2c(Gc)
    R = Uc @ torch.diag_embed(Sc.to(Gc.dtype)) @ Vc.conj().transpose(1, 2)
    assert (R - Gc).abs().max().item() < 1e-14
    mats = [np.random.default_rng(n).standard_normal((n, n)) for n in (8, 16, 32)]
    p = sweep.Packed(mats)
    res = sweep.kog_sweep_batch(p, sort=True)
    for M, s in zip(mats, p.unpack_sigma(res["sigma"])):
        assert np.allclose(s, np.linalg.svd(M, compute_uv=False), rtol=1e-12, atol=1e-12)
    tall, sweeps = sweep.svd_rect([np.random.default_rng(1).standard_normal((40, 16))])
    assert sweeps[0] > 0 and tall[0][0].shape == (40, 16)
