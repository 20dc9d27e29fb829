"""GPU parity of the complex 2x2 SVD (Sect. 3.4): U, S, V, the (e,f) pairs and the info
words bit for bit against the oracle.

Cases: every zero pattern of the complex elements x edge values in either part; the
complex recipe (narrow exponents, triangular, mixed real/imaginary elements, single row,
column and diagonal patterns, purely real and purely imaginary matrices) at 2^20 + 37
matrices (several tiles and a ragged tail), at its full size 2^22 on sampled outputs,
and with wide exponent ranges; batch sizes 0, 1, 257; non-finite inputs.
"""
import numpy as np
import pytest

from paper_2407_13116_amd import inputs

pytestmark = pytest.mark.gpu
CDT = [np.complex128, np.complex64]


def _gpu(G):
    import torch

    from paper_2407_13116_amd import api

    Gd = torch.from_numpy(np.ascontiguousarray(G)).cuda()
    U, S, V, f, e, info = api.ksvd2c(Gd, with_pairs=True)
    torch.cuda.synchronize()
    return {"U": U.cpu().numpy(), "S": S.cpu().numpy(), "V": V.cpu().numpy(),
            "f": f.cpu().numpy(), "e": e.cpu().numpy(), "info": info.cpu().numpy()}


def _flat(a):
    """[B, ...] as [B, m] of real values (complex parts interleaved)."""
    a = np.ascontiguousarray(a)
    if np.iscomplexobj(a):
        a = a.view(a.real.dtype)
    return a.reshape(len(a), -1)


def _assert_same(got, want, idx=None, label=""):
    """Bit for bit, NaNs only required to coincide in position."""
    for k in ("U", "S", "V", "f", "e", "info"):
        a = _flat(got[k] if idx is None else got[k][idx])
        b = _flat(want[k])
        assert a.shape == b.shape, (label, k, a.shape, b.shape)
        if a.dtype.kind == "f":
            na, nb = np.isnan(a), np.isnan(b)
            assert np.array_equal(na, nb), (label, k, "NaN positions differ")
            ui = np.uint64 if a.dtype == np.float64 else np.uint32
            diff = (a.view(ui) != b.view(ui)) & ~na
        else:
            diff = a != b
        bad = np.nonzero(diff.any(axis=1))[0]
        assert bad.size == 0, (label, k, bad.size, bad[:5].tolist())


@pytest.mark.parametrize("cdt", CDT)
def test_complex_special_set_bitwise(orc, cdt):
    G = inputs.complex_special_set(cdt, per_type=2048)
    _assert_same(_gpu(G), orc.ksvd2c(G), label=f"special {cdt.__name__}")


@pytest.mark.parametrize("cdt", CDT)
@pytest.mark.parametrize("emax", [20, 500])
def test_complex_recipe_ragged_bitwise(orc, cdt, emax):
    e = emax if cdt == np.complex128 else min(emax, 60)
    G = inputs.complex_batch(cdt, seed=41, B=(1 << 20) + 37, emax=e)
    _assert_same(_gpu(G), orc.ksvd2c(G), label=f"2^20+37 {cdt.__name__} e{e}")


@pytest.mark.parametrize("cdt", CDT)
def test_complex_full_size_sampled_bitwise(orc, cdt):
    G = inputs.complex_batch(cdt)
    got = _gpu(G)
    B = len(G)
    rng = np.random.default_rng(97)
    idx = np.unique(np.concatenate([rng.integers(0, B, 1 << 15), np.arange(B - 500, B)]))
    _assert_same(got, orc.ksvd2c(G[idx]), idx=idx, label=f"2^22 sampled {cdt.__name__}")
    assert np.all(np.isfinite(got["U"])) and np.all(np.isfinite(got["V"]))
    assert np.all(got["S"][:, 0] >= got["S"][:, 1])


@pytest.mark.parametrize("n", [0, 1, 257])
def test_complex_small_batches(orc, n):
    G = inputs.complex_batch(np.complex128, seed=43, B=max(n, 1))[:n]
    got = _gpu(G)
    if n:
        _assert_same(got, orc.ksvd2c(G), label=f"B={n}")
    else:
        assert all(v.size == 0 for v in got.values())


@pytest.mark.parametrize("cdt", CDT)
def test_complex_nonfinite(orc, cdt):
    G = np.ones((4, 2, 2), cdt)
    G[1, 0, 0] = complex(np.nan, 0)
    G[2, 1, 1] = complex(0, np.inf)
    G[3, 0, 1] = complex(-np.inf, 1)
    got = _gpu(G)
    _assert_same(got, orc.ksvd2c(G), label="nonfinite")
    assert (got["info"][1:] >> 15 & 1).all() and not (got["info"][0] >> 15 & 1)
