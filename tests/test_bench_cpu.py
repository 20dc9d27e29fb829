"""bench.py's contract pieces that need no GPU: the one-GPU refusal, the roofline
object, and the traffic figure read from the committed counter summary."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_roofline_object():
    import bench

    f64 = {"B": 1 << 24, "ms_kernel": 0.44, "GBs": 3500.0}
    r = bench.roofline(f64)
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r
    assert r["bound"] == "alu" and r["unit"] == "T VALU lane-ops/s"
    # the lane-operation peak from the unit counts and the clock: 256 CUs x 4 SIMDs x 16
    # lanes x 2.4 GHz, half the FP64 vector TFLOP/s (an FMA is two flops)
    assert r["peak"] == pytest.approx(39.3216) and r["peak"] == pytest.approx(78.6 / 2, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    # achieved = the algorithmic lane operations per launch over the launch time
    assert r["achieved"] == pytest.approx(700 * (1 << 24) / 0.44e-3 / 1e12)
    m = r["measured"]
    assert m is None or (m["valu_lane_ops_per_matrix"] > 0 and
                         m["issue_frac"] == pytest.approx(m["issued_T_lane_ops_per_s"] / r["peak"]))
    # traffic: the counter summary's figure when it was taken on these kernel sources and
    # this batch, else null; never a figure for another batch size
    assert r["traffic"] is None or r["traffic"] > 0
    assert bench.measured_traffic((1 << 24) + 1) is None


def test_unknown_profile_workload_lists_the_names():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--profile-workload",
                        "nope"], capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "fwd64" in r.stderr or "no GPU" in r.stderr


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_sigma_reference_against_exact(dtype):
    """The benchmark's vectorised double-word sigma reference (used for the whole-batch
    error histograms) against exact rationals + 320-bit mpmath on 1,800 matrices of the
    accuracy workload (all three families, the full exponent range), on zero patterns
    and on exactly singular matrices: relative difference below 2^-90 (sigma_2 = 0 is
    reproduced exactly)."""
    import mpmath

    import bench
    from paper_2407_13116_amd import inputs
    from sigma_ref import exact_sigmas

    g, lab = inputs.forward_sweep(dtype, B=1 << 17, with_labels=True)
    rng = np.random.default_rng(9)
    idx = np.concatenate([rng.choice(np.nonzero(lab == k)[0], 600, replace=False)
                          for k in range(3)])
    planes = [p[idx] for p in g]
    one, z = dtype(1.5), dtype(0)
    extra = [(one, z, z, z), (z, z, z, z), (one, one, one, one), (one, z, z, one),
             (z, one, one, z), (dtype(3), dtype(4), dtype(6), dtype(8))]
    planes = [np.concatenate([p, np.array([e[i] for e in extra], dtype)])
              for i, p in enumerate(planes)]
    m1h, m1l, E1, m2h, m2l, E2 = bench.sigma_ref(*planes)
    with mpmath.workprec(320):
        for k in range(planes[0].size):
            s1, s2 = exact_sigmas(*(p[k] for p in planes))
            for s, mh, ml, E in ((s1, m1h, m1l, E1), (s2, m2h, m2l, E2)):
                got = mpmath.ldexp(mpmath.mpf(float(mh[k])) + mpmath.mpf(float(ml[k])), int(E[k]))
                if s == 0:
                    assert mh[k] == 0 and ml[k] == 0, k
                else:
                    assert abs(got - s) / s < mpmath.mpf(2) ** -90, (k, float(got), float(s))


def test_sigma_error_histogram_counts():
    """The histogram of the benchmark places sigma values rounded to nearest at <= 1 eps
    and values one ulp further off above 1 eps, family by family."""
    import bench

    g = [np.array([3.0, 1.0]), np.array([0.0, 0.0]), np.array([0.0, 1.0]),
         np.array([4.0, 1.0])]          # diag(3, 4) (sigma 4, 3) and [[1 1];[0 1]]
    m1h, m1l, E1, m2h, m2l, E2 = bench.sigma_ref(*g)
    assert list(E1) == [3, 1] and m1h[0] == 0.5 and m2h[0] == 0.75   # 4 and 3 exactly
    f1, e1 = 2 * m1h, E1 - 1            # the (e, f) form, f in [1, 2): rounded to nearest
    f2, e2 = 2 * m2h, E2 - 1
    f2[1] = np.nextafter(f2[1], 2.0)    # sigma_2 of the second matrix one ulp up
    host = {"f1": f1, "e1": e1, "f2": f2, "e2": e2}
    h = bench.sigma_error_histogram(g, host, np.array([0, 1], np.int8), np.float64)
    assert h["sigma1"]["general"]["hist"]["<=1"] == 1 and h["sigma1"]["general"]["max"] == 0
    assert h["sigma1"]["upper_triangular"]["hist"]["<=1"] == 1
    assert h["sigma2"]["general"]["max"] == 0.0
    assert 1.0 < h["sigma2"]["upper_triangular"]["max"] <= 4.0
    assert h["sigma2"]["upper_triangular"]["hist"]["<=1"] == 0
