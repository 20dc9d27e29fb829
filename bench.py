#!/usr/bin/env python3
"""Benchmark of the batched enhanced Kogbetliantz 2x2 SVD on one MI355X.

One step = one pass of the forward hot path (classification, prescaling, the
URV factorisation, the triangular SVD, assembly and backscaling) over the
accuracy/throughput workload: 2^24 binary64 2x2 matrices with entries
+-m 2^e, e uniform in [-1000, 1000], 10% upper triangular, 1% near-singular,
resident in HBM as four planes before the timed region starts.

Printed (one JSON line): the headline rate (FP64 forward, 2x2 SVDs/s), the
roofline of the forward kernel (HIP events on the launch stream), the oracle on
the host cores as the CPU baseline, and in "extra": FP32 forward, forward +
backward (the differentiable workload, 2^22 matrices, both precisions), the
sweep throughput when available, and the max relative error of sigma_2 in units
of eps on a sample (by input class).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("2x2 SVDs/sec (fwd, fwd+bwd) FP64/FP32; %HBM roofline; max rel err σ2 (ulp)")
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_FWD = {np.float64: 92, np.float32: 52}      # algorithmic bytes per matrix (in + out)
BYTES_FWDBWD = {np.float64: 112 + 192, np.float32: 56 + 96}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extra", action="store_true", help="headline only")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_loop(fn, steps, warmup):
    """Warm up, then time exactly `steps` calls: wall clock between two synchronisations,
    and HIP events recorded on the launch stream around the same region."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall / steps * 1e3, ev0.elapsed_time(ev1) / steps


def fwd_case(dtype, steps, warmup):
    import torch

    from paper_2407_13116_amd import api, inputs

    g = inputs.forward_sweep(dtype)
    d = [torch.from_numpy(x).cuda() for x in g]
    out = api.ksvd2_batch(*d, plain=False)
    torch.cuda.synchronize()
    ms_wall, ms_ev = timed_loop(lambda: api.ksvd2_batch(*d, plain=False, out=out), steps, warmup)
    B = g[0].size
    res = {"B": B, "ms_wall": ms_wall, "ms_kernel": ms_ev, "rate": B / (ms_wall * 1e-3)}
    res["GBs"] = B * BYTES_FWD[dtype] / (ms_ev * 1e-3) / 1e9
    host = {k: v.cpu().numpy() for k, v in out.items()}
    del d, out
    torch.cuda.empty_cache()
    return res, g, host


def fwdbwd_case(dtype, steps, warmup):
    import torch

    from paper_2407_13116_amd import api, inputs

    G, dS, dU, dV, _ = inputs.diff_batch(dtype)
    t = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (G, dS, dU, dV)]

    def step():
        U, S, V = api.svd2x2_raw(t[0])
        return api.svd2x2_backward(U, S, V, t[1], t[2], t[3])

    ms_wall, ms_ev = timed_loop(step, max(steps // 2, 5), warmup)
    B = G.shape[0]
    out = {"B": B, "ms_wall": ms_wall, "ms_kernel": ms_ev, "rate": B / (ms_wall * 1e-3),
           "GBs": B * BYTES_FWDBWD[dtype] / (ms_ev * 1e-3) / 1e9}
    del t
    torch.cuda.empty_cache()
    return out


def sigma2_error_sample(g, host, dtype, n=1500):
    """max relative error of sigma_2 (units of eps) on a sample, by input class, against
    a high-precision closed form (exact rationals + mpmath)."""
    from fractions import Fraction

    import mpmath

    eps = 2.0 ** (-53 if dtype == np.float64 else -24)
    B = g[0].size
    idx = np.random.default_rng(5).choice(B, n, replace=False)
    worst = {"triangular": 0.0, "general": 0.0}
    with mpmath.workprec(320):
        for i in idx:
            a, b, c, d = (Fraction(float(p[i])) for p in g)
            F = a * a + b * b + c * c + d * d
            D = a * d - c * b
            if F == 0:
                continue
            disc = F * F - 4 * D * D
            s1 = mpmath.sqrt((mpmath.mpf(F.numerator) / F.denominator
                              + mpmath.sqrt(mpmath.mpf(disc.numerator) / disc.denominator)) / 2)
            s2 = abs(mpmath.mpf(D.numerator) / D.denominator) / s1
            got = mpmath.ldexp(mpmath.mpf(float(host["f2"][i])), int(host["e2"][i]))
            re = 0.0 if s2 == 0 and got == 0 else float(abs(got - s2) / s2 / eps) if s2 else float("inf")
            key = "triangular" if b == 0 else "general"
            worst[key] = max(worst[key], re)
    return worst


def cpu_baseline(seconds):
    import oracle
    from paper_2407_13116_amd import inputs

    oracle.build(force=False)
    nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    g = inputs.forward_sweep(np.float64, B=1 << 22)
    oracle.ksvd2(*(p[:4096] for p in g), nthreads=nthreads, plain=False)   # warm
    done, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        oracle.ksvd2(*g, nthreads=nthreads, plain=False)
        done += g[0].size
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "2x2 SVDs/s", "cores": nthreads, "kind": "oracle",
            "sample": f"first 2^22 matrices of the FP64 2^24 workload, repeated for ~{seconds:.0f} s "
                      f"({done} SVDs in {dt:.1f} s), OpenMP static schedule"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the batched 2x2 "
              "SVD shards by matrix with no communication, and multi-GPU runs are not part "
              "of this build.", file=sys.stderr)
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "no GPU"
    log("[bench] FP64 forward, 2^24 matrices")
    f64, g64, h64 = fwd_case(np.float64, args.steps, args.warmup)
    log(f"[bench] f64: {f64}")
    res = {
        "metric": METRIC,
        "value": f64["rate"],
        "unit": "2x2 SVDs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["ms_wall"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "forward accuracy/throughput sweep: 2^24 FP64 2x2 matrices, "
                               "entries +-m 2^e with e uniform in [-1000,1000], 10% upper "
                               "triangular, 1% near-singular, SoA planes resident in HBM",
                   "batch": f64["B"]},
        "roofline": {"bound": "hbm", "achieved": f64["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": f64["GBs"] / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_fwd_soa<double>", "avg_kernel_ms": f64["ms_kernel"],
                     "bytes_per_matrix": BYTES_FWD[np.float64]},
    }
    extra = {}
    if not args.no_extra:
        log("[bench] FP32 forward, 2^24 matrices")
        f32, g32, h32 = fwd_case(np.float32, args.steps, args.warmup)
        extra["fwd_f32"] = {"rate": f32["rate"], "ms_per_launch": f32["ms_kernel"],
                            "GBs": f32["GBs"], "hbm_frac": f32["GBs"] / HBM_PEAK_GBS}
        for dt, name in ((np.float64, "fwdbwd_f64"), (np.float32, "fwdbwd_f32")):
            log(f"[bench] {name}, 2^22 matrices")
            fb = fwdbwd_case(dt, args.steps, args.warmup)
            extra[name] = {"rate": fb["rate"], "ms_per_step": fb["ms_kernel"], "GBs": fb["GBs"],
                           "hbm_frac": fb["GBs"] / HBM_PEAK_GBS}
        log("[bench] sigma_2 accuracy sample")
        extra["max_rel_err_sigma2_ulp"] = {"f64": sigma2_error_sample(g64, h64, np.float64),
                                           "f32": sigma2_error_sample(g32, h32, np.float32),
                                           "unit": "eps (2^-53 / 2^-24)",
                                           "sample": "1,500 matrices per precision"}
    res["extra"] = extra
    if not args.no_cpu:
        log("[bench] oracle CPU baseline")
        res["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
