"""GPU parity of the variant for a hypot that is not correctly rounded (Algorithm tf, its
branch for that case): every output bit for bit against the oracle's variant.

Cases: the fast hypot itself (random exponent gaps, subnormals, zeros, the overflow
edge); every zero pattern x edge values; both sub-branches of the tan(2 phi) formula; the
accuracy/throughput recipe at 2^20 + 37 matrices (several tiles and a ragged tail); the
full 2^24 batch in the benchmark's launch configuration on sampled outputs; batch sizes
0, 1 and 257.
"""
import numpy as np
import pytest

from gpu_util import assert_bitwise, gpu_ksvd2, to_dev
from paper_2407_13116_amd import inputs
from test_oracle_fast import _tri

pytestmark = pytest.mark.gpu
DTYPES = [np.float64, np.float32]


@pytest.mark.parametrize("dtype", DTYPES)
def test_device_fast_hypot_bitwise(orc, dtype):
    from paper_2407_13116_amd import api

    rng = np.random.default_rng(23)
    f = np.finfo(dtype)
    n = 1 << 18
    e1 = rng.integers(f.minexp - f.nmant, f.maxexp, n)
    e2 = e1 - rng.integers(0, 70, n)
    x = np.ldexp(1 + rng.random(n), e1).astype(dtype)
    y = np.ldexp(1 + rng.random(n), np.maximum(e2, f.minexp - f.nmant)).astype(dtype)
    ks = rng.integers(1, 1 << f.nmant, (2, 4096))
    xs = (ks[0] * np.float64(f.smallest_subnormal)).astype(dtype)
    ys = (ks[1] * np.float64(f.smallest_subnormal)).astype(dtype)
    xe = np.array([f.max, 1, 0, 0, f.max / 2, 3, np.inf, 1], dtype)
    ye = np.array([1, f.max, 0, 5, f.max / 2, 4, 1, -np.inf], dtype)
    # ratios in [2^-28, 2^-10]: 1 + r^2 just above 1, where the root is formed directly
    # (every s = 1 + k 2^-52 with small k, odd and even), against (t, 1) and scaled pairs
    t = np.ldexp(1 + rng.random(20000), -rng.integers(11, 29, 20000)).astype(dtype)
    hi = np.ldexp(1 + rng.random(20000), rng.integers(-60, 60, 20000)).astype(dtype)
    X = np.concatenate([x, xs, xe, -x[:1000], t, hi * t, np.ones_like(t)])
    Y = np.concatenate([y, ys, ye, y[:1000], np.ones_like(t), hi, -t])
    xd, yd = to_dev(X, Y)
    got = api.hypot(xd, yd, fast=True).cpu().numpy()
    want = orc.hypot(X, Y, fast=True)
    assert_bitwise({"h": got}, {"h": want}, label="fast hypot vs oracle")


@pytest.mark.parametrize("dtype", DTYPES)
def test_fast_special_set_bitwise(orc, dtype):
    g = inputs.special_set(dtype, per_type=4096)
    assert_bitwise(gpu_ksvd2(g, fast=True), orc.ksvd2(*g, fast=True),
                   label=f"fast special set {dtype.__name__}")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("big_first", [True, False], ids=["r11>r12", "r11<=r12"])
def test_fast_tan2phi_branches_bitwise(orc, dtype, big_first):
    rng = np.random.default_rng(40 + big_first)
    emax = 400 if dtype == np.float64 else 40
    G = _tri(rng, 20000, dtype, emax, big_first)
    g = tuple(np.ascontiguousarray(G[:, k]) for k in range(4))
    assert_bitwise(gpu_ksvd2(g, fast=True), orc.ksvd2(*g, fast=True),
                   label=f"fast tan2phi {dtype.__name__} {big_first}")


@pytest.mark.parametrize("dtype", DTYPES)
def test_fast_recipe_ragged_bitwise(orc, dtype):
    g = inputs.forward_sweep(dtype, B=(1 << 20) + 37)
    assert_bitwise(gpu_ksvd2(g, fast=True), orc.ksvd2(*g, fast=True),
                   label=f"fast 2^20+37 {dtype.__name__}")


@pytest.mark.parametrize("dtype", DTYPES)
def test_fast_full_size_sampled_bitwise(orc, dtype):
    g = inputs.forward_sweep(dtype)
    got = gpu_ksvd2(g, fast=True)
    B = g[0].size
    rng = np.random.default_rng(98)
    idx = np.unique(np.concatenate([rng.integers(0, B, 1 << 16), np.arange(B - 1000, B)]))
    want = orc.ksvd2(*(p[idx] for p in g), fast=True)
    assert_bitwise(got, want, idx=idx, label=f"fast 2^24 sampled {dtype.__name__}")
    assert np.all(np.isfinite(got["cu"])) and np.all(np.isfinite(got["sv"]))


@pytest.mark.parametrize("n", [0, 1, 257])
def test_fast_small_batches(orc, n):
    g = inputs.forward_sweep(np.float64, B=max(n, 1), seed=6)
    g = tuple(p[:n] for p in g)
    got = gpu_ksvd2(g, fast=True)
    if n:
        assert_bitwise(got, orc.ksvd2(*g, fast=True), label=f"fast B={n}")
    else:
        assert all(v.size == 0 for v in got.values())
