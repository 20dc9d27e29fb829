"""bench.py's contract pieces that need no GPU: the one-GPU refusal, the roofline
object, and the traffic figure read from the committed counter summary."""
import os
import subprocess
import sys

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
