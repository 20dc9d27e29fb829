"""GPU parity of the batched 2x2 SVD: every output bit for bit against the oracle.

Cases: the 65,536-matrix forward workload with its zero patterns; every zero pattern x
edge values (signed zeros, subnormals, mu, nu, ties); the accuracy/throughput recipe at
2^20 + 37 matrices (several tiles and a ragged tail) for both precisions, and at its full
size 2^24 in the launch configuration the benchmark times, checked on sampled outputs;
batch sizes 0, 1, 255, 257, and 2^28 + 4,099 (more than one launch); non-finite inputs;
the autograd layout; the device hypot.
"""
import numpy as np
import pytest

from exact_ref import exact_hypot
from gpu_util import assert_bitwise, gpu_ksvd2, to_dev
from paper_2407_13116_amd import inputs

pytestmark = pytest.mark.gpu
DTYPES = [np.float64, np.float32]


def test_forward_small_workload_bitwise(orc):
    g = inputs.forward_small(seed=1)
    want = orc.ksvd2(*g)
    got = gpu_ksvd2(g)
    assert_bitwise(got, want, label="forward_small f64")


@pytest.mark.parametrize("dtype", DTYPES)
def test_special_set_bitwise(orc, dtype):
    g = inputs.special_set(dtype, per_type=4096)
    want = orc.ksvd2(*g)
    got = gpu_ksvd2(g)
    assert_bitwise(got, want, label=f"special set {dtype.__name__}")


@pytest.mark.parametrize("dtype", DTYPES)
def test_sweep_recipe_ragged_bitwise(orc, dtype):
    g = inputs.forward_sweep(dtype, B=(1 << 20) + 37)
    want = orc.ksvd2(*g)
    got = gpu_ksvd2(g)
    assert_bitwise(got, want, label=f"2^20+37 {dtype.__name__}")


@pytest.mark.parametrize("dtype", DTYPES)
def test_full_size_sampled_bitwise(orc, dtype):
    """2^24 matrices, one launch as the benchmark runs it; 2^16 sampled outputs plus the
    last 1,000 are recomputed by the oracle one by one."""
    g = inputs.forward_sweep(dtype)
    got = gpu_ksvd2(g)
    B = g[0].size
    rng = np.random.default_rng(99)
    idx = np.unique(np.concatenate([rng.integers(0, B, 1 << 16), np.arange(B - 1000, B)]))
    want = orc.ksvd2(*(p[idx] for p in g))
    assert_bitwise(got, want, idx=idx, label=f"2^24 sampled {dtype.__name__}")
    # whole-batch properties
    assert np.all(np.isfinite(got["cu"])) and np.all(np.isfinite(got["sv"]))
    f1, f2 = got["f1"], got["f2"]
    assert np.all((f1 >= 1) & (f1 < 2))
    assert np.all(((f2 >= 1) & (f2 < 2)) | ((f2 == 0) & (got["e2"] == 0)))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("seed", [101, 202, 303])
def test_more_seeds_bitwise(orc, dtype, seed):
    """The accuracy/throughput recipe with other seeds, 2^19 + 11 matrices each, and its
    exponent range narrowed to a quarter (fewer exponent-gap exits, more full hypots)."""
    g = inputs.forward_sweep(dtype, seed=seed, B=(1 << 19) + 11)
    assert_bitwise(gpu_ksvd2(g), orc.ksvd2(*g), label=f"seed {seed} {dtype.__name__}")
    q = tuple(np.ldexp(m, e // 4).astype(dtype) for m, e in (np.frexp(p) for p in g))
    assert_bitwise(gpu_ksvd2(q), orc.ksvd2(*q), label=f"seed {seed} narrow {dtype.__name__}")


@pytest.mark.parametrize("n", [1, 2, 255, 256, 257])
def test_small_batches(orc, n):
    g = inputs.forward_sweep(np.float64, B=n, seed=5)
    assert_bitwise(gpu_ksvd2(g), orc.ksvd2(*g), label=f"B={n}")


def test_empty_batch_is_noop():
    import torch

    from paper_2407_13116_amd import api

    e = torch.empty(0, dtype=torch.float64, device="cuda")
    out = api.ksvd2_batch(e, e, e, e)
    torch.cuda.synchronize()
    assert all(v.numel() == 0 for v in out.values())


@pytest.mark.parametrize("dtype", DTYPES)
def test_nonfinite_inputs(orc, dtype):
    g = [np.array([1, np.nan, 0, np.inf, 2], dtype), np.ones(5, dtype), np.ones(5, dtype),
         np.array([1, 1, -np.inf, 1, 3], dtype)]
    got = gpu_ksvd2(g)
    want = orc.ksvd2(*g)
    assert_bitwise(got, want, label="nonfinite")
    assert list((got["info"] >> 15) & 1) == [0, 1, 1, 1, 0]


@pytest.mark.parametrize("dtype", DTYPES)
def test_autograd_layout_matches_soa(orc, dtype):
    import torch

    from paper_2407_13116_amd import api

    g = inputs.forward_sweep(dtype, B=50001, seed=8)
    G = inputs.mats_from_soa(*g)
    U, S, V, info = api.svd2x2_raw(to_dev(G)[0], with_info=True)
    torch.cuda.synchronize()
    want = orc.ksvd2(*g)
    Uo, Vo = orc.full_uv(want)
    assert np.array_equal(info.cpu().numpy(), want["info"])
    for got_t, ref in ((U, Uo), (V, Vo)):
        got_n = got_t.cpu().numpy().astype(np.float64)
        assert np.array_equal(got_n, ref)   # values (signs of zeros aside)
    Sn = S.cpu().numpy()
    for k, col in (("s1", 0), ("s2", 1)):
        assert_bitwise({k: np.ascontiguousarray(Sn[:, col])}, {k: want[k]}, label="S " + k)


@pytest.mark.parametrize("dtype", DTYPES)
def test_device_hypot(orc, dtype):
    import torch

    from paper_2407_13116_amd import api

    rng = np.random.default_rng(17)
    f = np.finfo(dtype)
    n = 1 << 18
    e1 = rng.integers(f.minexp - f.nmant, f.maxexp, n)
    e2 = e1 - rng.integers(0, 70, n)
    x = np.ldexp(1 + rng.random(n), e1).astype(dtype)
    y = np.ldexp(1 + rng.random(n), np.maximum(e2, f.minexp - f.nmant)).astype(dtype)
    # subnormal pairs, exact Pythagorean ties, Lemma nu, zeros, overflow edge
    ks = rng.integers(1, 1 << f.nmant, (2, 4096))
    xs = (ks[0] * np.float64(f.smallest_subnormal)).astype(dtype)
    ys = (ks[1] * np.float64(f.smallest_subnormal)).astype(dtype)
    from test_oracle_hypot_ef import _pythagorean_midpoints
    p = f.nmant + 1
    trip = _pythagorean_midpoints(p, 512, rng)
    xt = np.array([np.ldexp(t[0], s) for t in trip for s in (0, -30, 40)], dtype)
    yt = np.array([np.ldexp(t[1], s) for t in trip for s in (0, -30, 40)], dtype)
    xe = np.array([f.max, 1, 0, 0, f.max, f.max / 2, 3], dtype)
    ye = np.array([1, f.max, 0, 5, f.max, f.max / 2, 4], dtype)
    X = np.concatenate([x, xs, xt, xe, -x[:1000]])
    Y = np.concatenate([y, ys, yt, ye, y[:1000]])
    xd, yd = to_dev(X, Y)
    got = api.hypot(xd, yd).cpu().numpy()
    want = orc.hypot(X, Y)
    assert_bitwise({"h": got}, {"h": want}, label="hypot vs oracle")
    # and the exact reference on a subset (independent of both)
    for i in list(range(0, n, 997)) + list(range(n, X.size)):
        assert got[i] == exact_hypot(X[i], Y[i], dtype), (X[i], Y[i])


@pytest.mark.parametrize("dtype", DTYPES)
def test_batch_past_one_launch(orc, dtype):
    """A batch of 2^28 + 4,099 matrices: more than one launch (each covers at most 2^28
    matrices with 32-bit offsets).  Inputs drawn on the device; outputs around the launch
    boundary, the last 1,000 and 2^14 random ones recomputed by the oracle."""
    import torch

    from paper_2407_13116_amd import api

    tdt = torch.float64 if dtype == np.float64 else torch.float32
    B = (1 << 28) + 4099
    gen = torch.Generator(device="cuda").manual_seed(2828)
    planes = [torch.randn(B, dtype=tdt, device="cuda", generator=gen) for _ in range(4)]
    out = api.ksvd2_batch(*planes, plain=False)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([np.arange((1 << 28) - 3000, (1 << 28) + 3000),
                                    np.arange(B - 1000, B), rng.integers(0, B, 1 << 14)]))
    it = torch.from_numpy(idx).cuda()
    g = [p.index_select(0, it).cpu().numpy() for p in planes]
    got = {k: v.index_select(0, it).cpu().numpy() for k, v in out.items()}
    del planes, out
    torch.cuda.empty_cache()
    assert_bitwise(got, orc.ksvd2(*g), label=f"2^28+4099 {dtype.__name__}")


def test_device_hypot_binary32_dense(orc):
    """The binary32 hypot (binary32 arithmetic with a certified candidate, the binary64
    route for the rest) bit for bit against the oracle on 2^24 random pairs across
    exponent gaps 0..20 (the gap exit is at 13), on 2^20 pairs built next to rounding
    midpoints (x random, y = RN(sqrt(m^2 - x^2)) and its neighbours for a midpoint m),
    next to the overflow threshold, around roots of 2 after scaling, and with
    subnormal larger arguments."""
    import torch

    from paper_2407_13116_amd import api

    rng = np.random.default_rng(23)
    f = np.finfo(np.float32)
    n = 1 << 24
    e1 = rng.integers(-125, 127, n)
    x = np.ldexp(1 + rng.random(n), e1).astype(np.float32)
    y = np.ldexp(1 + rng.random(n), e1 - rng.integers(0, 21, n)).astype(np.float32)
    # next to midpoints: m = float + half an ulp (in binary64, exact), x below m
    k = 1 << 18
    mant = (1 + rng.integers(0, 1 << 23, k) * 2.0 ** -23)
    m = (mant + 2.0 ** -24) * np.ldexp(1.0, rng.integers(-100, 100, k))
    xm = (m * rng.random(k)).astype(np.float32).astype(np.float64)
    ym = np.sqrt(np.maximum(m * m - xm * xm, 0)).astype(np.float32)
    ymm = [ym, np.nextafter(ym, np.float32(np.inf)), np.nextafter(ym, np.float32(0))]
    xs = np.concatenate([xm.astype(np.float32)] * 3)
    ys = np.concatenate(ymm)
    # overflow edge and roots of 2 after scaling (A^2 + B^2 near 4)
    big = np.array([f.max, np.nextafter(f.max, 0), 2.0 ** 127, 1.9 * 2.0 ** 127], np.float32)
    xo = np.repeat(big, 256)
    yo = (np.ldexp(rng.random(xo.size), 127 - rng.integers(0, 16, xo.size))).astype(np.float32)
    t = (2 - rng.random(1 << 16) * 2.0 ** -10).astype(np.float32)          # A just below 2
    xr = t
    yr = (rng.random(t.size) * 2.0 ** -6).astype(np.float32)
    sub = (rng.integers(1, 1 << 23, (2, 1 << 14)) * np.float64(f.smallest_subnormal)).astype(np.float32)
    X = np.concatenate([x, xs, xo, xr, sub[0], -x[:4096]])
    Y = np.concatenate([y, ys, yo, yr, sub[1], y[:4096]])
    xd, yd = to_dev(X, Y)
    got = api.hypot(xd, yd).cpu().numpy()
    torch.cuda.synchronize()
    want = orc.hypot(X, Y)
    assert_bitwise({"h": got}, {"h": want}, label="binary32 hypot vs oracle")
