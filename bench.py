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
FP64_VECTOR_TFLOPS = 78.6      # 256 CU x 64 lanes x 2.4 GHz x 2 (an FMA counts twice)
# VALU lane-operation peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave64 instruction
# occupies a SIMD for 4 cycles; binary64 FMA at this full rate is the 78.6 TFLOP/s above)
VALU_LANE_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic work per matrix of the forward method (main class-15 path), in VALU lane
# operations: about 8 correctly rounded hypot (~45 each in FP64), 18 IEEE divisions (~13),
# ~45 add/mul/fma, the double-word EXT block and ~25 exponent operations -> ~700 per FP64
# matrix (~400 for FP32, hypot evaluated in binary64)
ALG_VALU_SLOTS = {np.float64: 700, np.float32: 400}
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "pmc_traffic_k_fwd_soa_f64.md")
VALU_PROFILE = os.path.join(ROOT, "profiles", "pmc_valu_2x2_kernels.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2407_13116_amd", "csrc", f)
                  for f in ("ksvd2_device.hpp", "ksvd2_kernels.hip", "abi_common.hpp")]
BYTES_FWD = {np.float64: 92, np.float32: 52}      # algorithmic bytes per matrix (in + out)
BYTES_FWDBWD = {np.float64: 112 + 192, np.float32: 56 + 96}
BYTES_BWD = {np.float64: 192, np.float32: 96}     # backward alone ([B,2,2] layout)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    # untimed steps after the clock-settling phase (settle())
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extra", action="store_true", help="headline only")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--profile-workload", default=None,
                    help="run one named workload for a profiler and exit (see "
                         "PROFILE_WORKLOADS)")
    ap.add_argument("--reps", type=int, default=3, help="launches after the first, with "
                    "--profile-workload")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


SETTLE_S = 0.25   # the GPU clock ramps up over the first ~25 ms of back-to-back launches


def settle(fn, seconds=SETTLE_S):
    """Run fn back to back for at least `seconds` (untimed, before the warm-up steps) so
    that the timed steps do not sit inside the clock ramp; returns the calls made."""
    import torch

    calls, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(4):
            fn()
        calls += 4
        torch.cuda.synchronize()
    return calls


def timed_loop(fn, steps, warmup, per_launch=None):
    """Settle the clock, do `warmup` untimed calls, then time exactly `steps` calls: wall
    clock between two synchronisations, and HIP events recorded on the launch stream
    around the same region.  With a list as `per_launch`, an event is also recorded
    between consecutive calls and the durations of the timed calls (ms) are appended."""
    import torch

    settle(fn)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    evs[0].record()
    for i in range(steps):
        fn()
        if per_launch is not None or i == steps - 1:
            evs[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if per_launch is not None:
        per_launch.extend(evs[i].elapsed_time(evs[i + 1]) for i in range(steps))
    return wall / steps * 1e3, evs[0].elapsed_time(evs[steps]) / steps


def fwd_case(dtype, steps, warmup, fast=False, per_launch=None):
    import torch

    from paper_2407_13116_amd import api, inputs

    g, lab = inputs.forward_sweep(dtype, with_labels=True)
    d = [torch.from_numpy(x).cuda() for x in g]
    out = api.ksvd2_batch(*d, plain=False, fast=fast)
    torch.cuda.synchronize()
    ms_wall, ms_ev = timed_loop(lambda: api.ksvd2_batch(*d, plain=False, out=out, fast=fast),
                                steps, warmup, per_launch)
    B = g[0].size
    res = {"B": B, "ms_wall": ms_wall, "ms_kernel": ms_ev, "rate": B / (ms_wall * 1e-3)}
    res["GBs"] = B * BYTES_FWD[dtype] / (ms_ev * 1e-3) / 1e9
    host = {k: v.cpu().numpy() for k, v in out.items()}
    host["labels"] = lab
    del d, out
    torch.cuda.empty_cache()
    return res, g, host


def complex_case(cdt, steps, warmup):
    """The complex 2x2 SVD (Sect. 3.4) of the 2^22-matrix complex recipe: G in, U, S, V
    out (64 + 144 = 208 / 104 algorithmic bytes per matrix in complex128 / complex64)."""
    import torch

    from paper_2407_13116_amd import api, inputs

    G = torch.from_numpy(inputs.complex_batch(cdt)).cuda()
    ms_wall, ms_ev = timed_loop(lambda: api.ksvd2c(G), steps, warmup)
    B = G.shape[0]
    per = 208 if cdt == np.complex128 else 104
    out = {"B": B, "rate": B / (ms_wall * 1e-3), "ms_per_launch": ms_ev,
           "GBs": B * per / (ms_ev * 1e-3) / 1e9}
    out["hbm_frac"] = out["GBs"] / HBM_PEAK_GBS
    del G
    torch.cuda.empty_cache()
    return out


def rect_case(dtype):
    """Rectangular inputs (Sect. 1): 256 tall 512 x 256 matrices, QR with column pivoting,
    the converged sweep on the triangular factors (persistent, modified modulus ordering,
    sorted), then U = Q [U_R; 0] and V = P V_R; one timed run after an untimed one."""
    import torch

    from paper_2407_13116_amd import inputs
    from paper_2407_13116_amd import sweep as sw

    pr = sw.PackedRect(inputs.rect_batch(dtype=dtype), dtype=dtype)
    sw.svd_rect_device(pr)
    pr.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = sw.svd_rect_device(pr)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    s = np.abs(out["sweeps"].cpu().numpy())
    res = {"matrices": len(pr.m), "shape": [int(pr.m[0]), int(pr.n[0])], "seconds": t,
           "matrices_per_s": len(pr.m) / t, "sweeps_mean": float(s.mean()),
           "converged": bool(np.all(out["sweeps"].cpu().numpy() > 0))}
    del pr, out
    torch.cuda.empty_cache()
    return res


def fwdbwd_case(dtype, steps, warmup):
    """Forward and backward of the differentiable workload through the
    torch.autograd.Function (api.svd2x2): G [B,2,2] -> (U, S, V), then torch.autograd.grad
    with the upstream gradients (dU, dS, dV), i.e. the adjoint kernel."""
    import torch

    from paper_2407_13116_amd import api, inputs

    G, dS, dU, dV, _ = inputs.diff_batch(dtype)
    t = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (G, dS, dU, dV)]
    t[0].requires_grad_(True)

    def step():
        U, S, V = api.svd2x2(t[0])
        return torch.autograd.grad((U, S, V), t[0], (t[2], t[1], t[3]))[0]

    ms_wall, ms_ev = timed_loop(step, max(steps // 2, 5), warmup)
    B = G.shape[0]
    out = {"B": B, "ms_wall": ms_wall, "ms_kernel": ms_ev, "rate": B / (ms_wall * 1e-3),
           "GBs": B * BYTES_FWDBWD[dtype] / (ms_ev * 1e-3) / 1e9}
    del t
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# sigma reference for the whole batch: double-word (about 104-bit) arithmetic,
# vectorised over numpy arrays, with exponents kept apart so that no product
# over- or underflows.  sigma_1 = (h1 + h2) / 2 with h1 = hypot(g11 + g22, g21 -
# g12) and h2 = hypot(g11 - g22, g12 + g21) (h1^2 = F + 2 det, h2^2 = F - 2 det
# with F = ||G||_F^2, so h1 + h2 = 2 sigma_1 for either sign of det, a sum of
# non-negative terms), sigma_2 = |det| / sigma_1 with det from exact products.
# Validated against exact rationals and mpmath in the CPU tests.

def _dw_two_sum(a, b):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def _dw_split(a):
    c = 134217729.0 * a          # 2^27 + 1 (operands are at most a few units here)
    hi = c - (c - a)
    return hi, a - hi


def _dw_two_prod(a, b):
    p = a * b
    ah, al = _dw_split(a)
    bh, bl = _dw_split(b)
    return p, ((ah * bh - p) + ah * bl + al * bh) + al * bl


def _dw_add(xh, xl, yh, yl):
    """AccurateDWPlusDW (Joldes, Muller, Popescu 2017, Algorithm 6): relative error
    below 3 2^-106 of the exact sum, also under cancellation."""
    sh, sl = _dw_two_sum(xh, yh)
    th, tl = _dw_two_sum(xl, yl)
    c = sl + th
    vh, vl = _dw_two_sum(sh, c)       # |sh| >= |c| may fail under cancellation: TwoSum
    w = tl + vl
    return _dw_two_sum(vh, w)


def _dw_mul(xh, xl, yh, yl):
    ph, pl = _dw_two_prod(xh, yh)
    pl = pl + (xh * yl + xl * yh)
    return _dw_two_sum(ph, pl)


def _dw_div(xh, xl, yh, yl):
    q = xh / yh
    ph, pl = _dw_two_prod(q, yh)
    r = ((xh - ph) - pl + xl - q * yl) / yh
    return _dw_two_sum(q, r)


def _dw_sqrt(xh, xl):
    with np.errstate(invalid="ignore", divide="ignore"):
        y = np.sqrt(xh)
        ph, pl = _dw_two_prod(y, y)
        r = ((xh - ph) - pl + xl) / (2.0 * y)
        r = np.where(y > 0, r, 0.0)
    return _dw_two_sum(y, r)


def sigma_ref(g11, g21, g12, g22):
    """Singular values of the 2x2 matrices [g11 g12; g21 g22] (float64 or float32
    planes) to about 2^-100 relative: (m1h, m1l, E1, m2h, m2l, E2) with sigma_i =
    (mih + mil) 2^Ei, or mih = mil = 0 for sigma_i = 0."""
    a, c, b, d = (np.asarray(x, np.float64) for x in (g11, g21, g12, g22))
    ax = np.maximum(np.maximum(np.abs(a), np.abs(b)), np.maximum(np.abs(c), np.abs(d)))
    _, emax = np.frexp(ax)
    sa, sb, sc, sd = (np.ldexp(x, -emax) for x in (a, b, c, d))   # exact but for tiny parts
    zero = np.zeros_like(sa)

    def hyp(xh, xl, yh, yl):
        x2 = _dw_mul(xh, xl, xh, xl)
        y2 = _dw_mul(yh, yl, yh, yl)
        return _dw_sqrt(*_dw_add(*x2, *y2))

    h1 = hyp(*_dw_two_sum(sa, sd), *_dw_two_sum(sc, -sb))
    h2 = hyp(*_dw_two_sum(sa, -sd), *_dw_two_sum(sb, sc))
    s1h, s1l = _dw_add(*h1, *h2)
    s1h, s1l = s1h * 0.5, s1l * 0.5
    # det = g11 g22 - g12 g21 from the exact products of the mantissas
    ma, ea = np.frexp(a)
    mb, eb = np.frexp(b)
    mc, ec = np.frexp(c)
    md, ed = np.frexp(d)
    p1h, p1l = _dw_two_prod(ma, md)
    p2h, p2l = _dw_two_prod(mb, mc)
    E1 = np.where(p1h != 0, ea + ed, -(1 << 30))
    E2 = np.where(p2h != 0, eb + ec, -(1 << 30))
    E = np.maximum(E1, E2)
    sh1, sh2 = np.maximum(E1 - E, -1100), np.maximum(E2 - E, -1100)
    dh, dl = _dw_add(np.ldexp(p1h, sh1), np.ldexp(p1l, sh1),
                     -np.ldexp(p2h, sh2), -np.ldexp(p2l, sh2))
    neg = dh < 0
    dh, dl = np.where(neg, -dh, dh), np.where(neg, -dl, dl)
    with np.errstate(invalid="ignore", divide="ignore"):
        qh, ql = _dw_div(dh, dl, s1h, s1l)
    ok = (s1h > 0) & (dh > 0)
    qh, ql = np.where(ok, qh, 0.0), np.where(ok, ql, 0.0)
    # normalise: sigma_1 = s1 2^emax, sigma_2 = q 2^(E - emax)
    _, f1 = np.frexp(s1h)
    _, f2 = np.frexp(qh)
    m1h, m1l = np.ldexp(s1h, -f1), np.ldexp(s1l, -f1)
    m2h, m2l = np.ldexp(qh, -f2), np.ldexp(ql, -f2)
    return (m1h, m1l, np.where(s1h > 0, emax + f1, 0), m2h, m2l,
            np.where(ok, E - emax + f2, 0))


def rel_err_ulps(f, e, mh, ml, me, eps):
    """|f 2^e - sigma| / sigma / eps for sigma = (mh + ml) 2^me (0/0 -> 0, x/0 -> inf)."""
    with np.errstate(invalid="ignore", over="ignore", divide="ignore"):
        t = np.ldexp(np.asarray(f, np.float64), np.clip(e - me, -1100, 1100))
        r = np.abs((t - mh) - ml) / mh / eps
    r = np.where(mh == 0, np.where(np.asarray(f) == 0, 0.0, np.inf), r)
    return r


ERR_EDGES = (1.0, 2.0, 4.0, 8.0, 16.0, 2.0 ** 10, 2.0 ** 26)


def sigma_error_histogram(g, host, labels, dtype, chunk=1 << 21):
    """Relative errors of sigma_1 and sigma_2 of the whole batch against sigma_ref, in
    units of eps, by family (general, upper triangular, near-singular): maximum and
    counts per bucket (<= 1, 2, 4, 8, 16, 2^10, 2^26 eps, more)."""
    eps = 2.0 ** (-53 if dtype == np.float64 else -24)
    names = ("general", "upper_triangular", "near_singular")
    buckets = [f"<={x:g}" for x in ERR_EDGES] + [f">{ERR_EDGES[-1]:g}"]
    out = {s: {n: {"max": 0.0, "hist": dict.fromkeys(buckets, 0)} for n in names}
           for s in ("sigma1", "sigma2")}
    B = g[0].size

    def errs(o):
        sl = slice(o, min(B, o + chunk))
        m1h, m1l, E1, m2h, m2l, E2 = sigma_ref(*(p[sl] for p in g))
        return (sl, rel_err_ulps(host["f1"][sl], host["e1"][sl], m1h, m1l, E1, eps),
                rel_err_ulps(host["f2"][sl], host["e2"][sl], m2h, m2l, E2, eps))

    # numpy releases the interpreter lock in its array operations: chunks in threads
    from concurrent.futures import ThreadPoolExecutor

    workers = max(1, min(8, (os.cpu_count() or 1) // 2))
    with ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(errs, range(0, B, chunk)))
    for sl, r1, r2 in parts:
        lab = labels[sl]
        for key, r in (("sigma1", r1), ("sigma2", r2)):
            idx = np.searchsorted(np.asarray(ERR_EDGES), r, side="left")
            for li, n in enumerate(names):
                sel = lab == li
                if not np.any(sel):
                    continue
                ent = out[key][n]
                ent["max"] = max(ent["max"], float(r[sel].max()))
                cnt = np.bincount(idx[sel], minlength=len(buckets))
                for bi, bname in enumerate(buckets):
                    ent["hist"][bname] += int(cnt[bi])
    return out


def sweep_case(mats, dtype, modes=("plain", "persistent", "graph"), max_sweeps=60, tune=True,
               traffic_profile=None):
    """Time one converged solve of a batch of square matrices per execution mode, with the
    modified modulus ordering, then once (persistent mode) with the round-robin and once
    with the dynamic ordering (the matrices are re-uploaded untimed before every run).
    ms_per_sweep is the solve's time over its largest sweep count (the batch finishes with
    its slowest matrix); with a committed counter summary of one sweep of this batch
    (traffic_profile), the HBM rate that sweep moves at this speed."""
    import torch

    from paper_2407_13116_amd import autotune
    from paper_2407_13116_amd import sweep as sw

    tdt = torch.float64 if dtype == np.float64 else torch.float32
    chosen = autotune.tune(mats, tdt) if tune else {}
    p = sw.Packed(mats, dtype=dtype)
    G0 = p.G.clone()
    # the schedule the autotuner picked per order bucket (0: n <= 64, 1: <= 128, 2: <= 256,
    # 3: <= 512): workgroup size, two steps per G pass, in-place pass, U/V chunk, tile rows
    res = {"tuned_knobs": {str(k): v for k, v in chosen.items()}}
    ws = None

    def solve(mode, ordering="modulus"):
        nonlocal ws
        p.G.copy_(G0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = sw.kog_sweep_batch(p, max_sweeps=max_sweeps, tol_factor=1.0, mode=mode,
                                 workspace=ws, sort=True, ordering=ordering)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        ws = out["workspace"]
        s = out["sweeps"].cpu().numpy()
        sa = np.abs(s)
        return out, {"seconds": t, "sweeps_mean": float(sa.mean()), "sweeps_max": int(sa.max()),
                     "converged": bool(np.all(s > 0)), "matrices_per_s": len(mats) / t,
                     "ms_per_sweep": t / max(int(sa.max()), 1) * 1e3}

    for mode in modes:
        if mode == "graph":
            solve(mode)                       # capture, then the timed replay
        out, res[mode] = solve(mode)
        log(f"[bench] sweep {mode}: {res[mode]}")
    if traffic_profile and "persistent" in modes:
        tb = measured_sweep_traffic(traffic_profile)
        if tb is not None:
            r = res["persistent"]
            gbs = tb / (r["ms_per_sweep"] * 1e-3) / 1e9
            r["hbm"] = {"measured_bytes_per_sweep": tb, "GBs": gbs, "frac": gbs / HBM_PEAK_GBS,
                        "source": os.path.relpath(traffic_profile, ROOT)}
    if "persistent" in modes:
        for name, ordering in (("persistent_round_robin_ordering", "round-robin"),
                               ("persistent_dynamic_ordering", "dynamic")):
            _, res[name] = solve("persistent", ordering)
            log(f"[bench] sweep persistent, {ordering}: {res[name]}")
        out, _ = solve("persistent")
    # the sigma gradient dG = U diag(dsigma) V^T of the last solve: 2 n^3 flops per matrix
    ds = torch.from_numpy(np.random.default_rng(17).standard_normal(int(p.n.sum())).astype(dtype)).cuda()
    fl = float(np.sum(2.0 * p.n.astype(np.float64) ** 3))
    ms_w, ms_ev = timed_loop(lambda: sw.sigma_grad(p, out["U"], out["V"], ds, workspace=ws), 10, 2)
    peak = FP64_VECTOR_TFLOPS if dtype == np.float64 else 157.3
    res["sigma_grad"] = {"ms": ms_ev, "TFLOPs": fl / (ms_ev * 1e-3) / 1e12,
                         "frac_mfma_peak": fl / (ms_ev * 1e-3) / 1e12 / peak,
                         "peak_TFLOPs": peak}
    log(f"[bench] sigma_grad: {res['sigma_grad']}")
    del p, G0
    torch.cuda.empty_cache()
    return res


SWEEP_SOURCES = [os.path.join(ROOT, "paper_2407_13116_amd", "csrc", f)
                 for f in ("kog_sweep.hip", "ksvd2_device.hpp", "abi_common.hpp")]
SWEEP_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "pmc_traffic_k_sw_persistent_f64_256x256.md")


def measured_sweep_traffic(path):
    """HBM bytes of one persistent sweep from a committed counter summary taken on the
    same kernel sources (else None)."""
    kv = _profile_values(path)
    try:
        if kv["kernel_source_sha256"] != kernel_source_hash(SWEEP_SOURCES):
            return None
        return float(kv["bytes_per_sweep"])
    except (KeyError, ValueError):
        return None


def kernel_source_hash(files=None):
    import hashlib

    h = hashlib.sha256()
    for f in files or KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _profile_values(path):
    """The `- key: value` lines of a committed counter summary."""
    kv = {}
    if not os.path.exists(path):
        return kv
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                kv[k.strip()] = v.strip().strip("`")
    return kv


def measured_traffic(batch):
    """HBM bytes per launch of the FP64 forward kernel from the committed rocprofv3
    --pmc summary (FETCH_SIZE scaled by the copy-kernel calibration factor, plus
    WRITE_SIZE), or None when that summary was taken on other kernel sources or another
    batch size."""
    kv = _profile_values(TRAFFIC_PROFILE)
    try:
        if kv["kernel_source_sha256"] != kernel_source_hash() or int(kv["batch"]) != batch:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measured_issue(batch, ms):
    """What the FP64 forward kernel issues, from the committed SQ counter summary (taken
    on the same kernel sources, else None): VALU instructions per wave (= lane operations
    per matrix, one matrix per lane) and binary64 flops per matrix (add, mul, 2 x fma,
    transcendental), turned into rates with this run's launch time."""
    kv = _profile_values(VALU_PROFILE)
    try:
        if kv["kernel_source_sha256"] != kernel_source_hash():
            return None
        valu = float(kv["fwd64_valu_per_wave"])
        flops = float(kv["fwd64_fp64_flops_per_matrix"])
    except (KeyError, ValueError):
        return None
    t = ms * 1e-3
    return {"valu_lane_ops_per_matrix": valu,
            "issued_T_lane_ops_per_s": valu * batch / t / 1e12,
            "issue_frac": valu * batch / t / 1e12 / VALU_LANE_PEAK_T,
            "fp64_flops_per_matrix": flops,
            "fp64_TFLOPs": flops * batch / t / 1e12,
            "fp64_frac": flops * batch / t / 1e12 / FP64_VECTOR_TFLOPS}


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
    # one thread on the first 2^18 matrices, ~2 s
    g1 = [p[:1 << 18] for p in g]
    d1, t1 = 0, time.perf_counter()
    while time.perf_counter() - t1 < 2.0:
        oracle.ksvd2(*g1, nthreads=1, plain=False)
        d1 += g1[0].size
    st = d1 / (time.perf_counter() - t1)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": done / dt, "unit": "2x2 SVDs/s", "cores": nthreads, "kind": "oracle",
            "sample": f"first 2^22 matrices of the FP64 2^24 workload, repeated for ~{seconds:.0f} s "
                      f"({done} SVDs in {dt:.1f} s), OpenMP static schedule",
            "single_thread_value": st, "cpu_model": model, "nproc": os.cpu_count()}


def oracle_beside(kind, seconds=2.0):
    """The oracle timed on a bounded sample of the same workload as a widened row's
    GPU case (host cores, OpenMP where the oracle has it)."""
    import oracle
    from paper_2407_13116_amd import inputs

    oracle.build(force=False)
    nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    if kind == "fast":
        g = [p[:1 << 20] for p in inputs.forward_sweep(np.float64, B=1 << 20)]
        done, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            oracle.ksvd2(*g, nthreads=nthreads, plain=False, fast=True)
            done += g[0].size
        unit, sample = "2x2 SVDs/s", "2^20 matrices of the FP64 forward workload, repeated"
    elif kind == "complex":
        G = inputs.complex_batch(np.complex128, B=1 << 20)
        done, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            oracle.ksvd2c(G, nthreads=nthreads)
            done += len(G)
        unit, sample = "complex 2x2 SVDs/s", "2^20 matrices of the complex128 recipe, repeated"
    else:
        mats = inputs.rect_batch(nmat=4)
        done, t0 = 0, time.perf_counter()
        for G in mats:
            oracle.svd_rect(G)
            done += 1
            if time.perf_counter() - t0 > seconds:
                break
        unit, sample = "matrices/s", f"{done} of the 512 x 256 FP64 matrices, one thread"
        nthreads = 1
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": unit, "cores": nthreads, "kind": "oracle",
            "sample": sample}


def roofline(f64):
    """The FP64 forward kernel is bound by VALU issue (its algorithmic bytes need only a
    third of HBM bandwidth at the measured rate): achieved = the method's algorithmic
    VALU lane operations per launch (700 per matrix) / the kernel's average duration (HIP
    events on its launch stream), against the chip's VALU lane-operation peak; beside it,
    what the kernel actually issues (counter summary) at this run's speed."""
    B, ms = f64["B"], f64["ms_kernel"]
    achieved = ALG_VALU_SLOTS[np.float64] * B / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": VALU_LANE_PEAK_T,
            "unit": "T VALU lane-ops/s", "frac": achieved / VALU_LANE_PEAK_T,
            "traffic": measured_traffic(B),
            "kernel": "k_fwd_soa<double>", "avg_kernel_ms": ms, "batch": B,
            "alg_valu_lane_ops_per_matrix": ALG_VALU_SLOTS[np.float64],
            "measured": measured_issue(B, ms),
            "hbm": {"achieved_GBs": f64["GBs"], "peak_GBs": HBM_PEAK_GBS,
                    "frac": f64["GBs"] / HBM_PEAK_GBS,
                    "alg_bytes_per_matrix": BYTES_FWD[np.float64]}}


def _class_batch(dtype, tri, B=1 << 22, seed=31):
    from paper_2407_13116_amd import inputs

    rng = np.random.default_rng(seed)
    G = inputs.signed_pow2_entries(rng, (B, 2, 2), -20, 20, dtype)
    if tri:
        G[:, 1, 0] = 0
    return inputs.soa_from_mats(G)


PROFILE_WORKLOADS = """
  fwd64 / fwd32     the 2^24-matrix forward workload (k_fwd_soa)
  fast64 / fast32   the same workload, the variant without a correctly rounded hypot
  cls15_64 / cls13_64 / cls15_32 / cls13_32
                    2^22 matrices of one class only (general, upper triangular; exponents
                    in [-20,20]): no lane divergence between classes, so the per-wave VALU
                    instruction count is the per-matrix path length of that class
  bwd64 / bwd32     the 2^22-matrix backward (k_bwd) after one forward (k_fwd_full)
  bwdsoa64 / bwdsoa32  the 2^22-matrix backward on the SoA planes (k_bwd_soa)
  cplx128 / cplx64  the 2^22-matrix complex 2x2 SVD (k_fwd_c)
  rect64            256 tall 512 x 256 FP64 matrices: k_qrcp, the sweep, k_qapply
  copy              a plain 1 GiB device-to-device copy (counter calibration: FETCH_SIZE
                    and WRITE_SIZE should each read 1 GiB)
  sweep4            one persistent sweep of the 256 x (n=256) FP64 workload
  sweep4rr          the same with the round-robin ordering
  sweep5 / sweep5f32  one persistent sweep of the 1,000 uneven orders 16-512 (FP64 / FP32)
  sgrad64 / sgrad32 the sigma-gradient U diag(dsigma) V^T of the 256 x (n=256) sweep
                    batch (FP64) or of the 1,000 uneven orders (FP32), after one sweep
"""


def profile_workload(w, reps):
    """One named workload for a profiling run (rocprofv3 --kernel-trace / --pmc): the
    kernel launched 1 + reps times on the same inputs, no timing, no JSON line."""
    import torch

    from paper_2407_13116_amd import api, inputs

    dev = lambda *a: [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in a]

    def fwd(g, fast=False):
        d = dev(*g)
        out = api.ksvd2_batch(*d, plain=False, fast=fast)
        for _ in range(reps):
            api.ksvd2_batch(*d, plain=False, out=out, fast=fast)

    if w in ("fwd64", "fwd32", "fast64", "fast32"):
        fwd(inputs.forward_sweep(np.float64 if w.endswith("64") else np.float32),
            fast=w.startswith("fast"))
    elif w.startswith("cls"):
        fwd(_class_batch(np.float64 if w.endswith("64") else np.float32,
                         tri=w.startswith("cls13")))
    elif w in ("bwd64", "bwd32"):
        G, dS, dU, dV, _ = inputs.diff_batch(np.float64 if w == "bwd64" else np.float32)
        t = dev(G, dS, dU, dV)
        U, S, V = api.svd2x2_raw(t[0])
        for _ in range(reps + 1):
            api.svd2x2_backward(U, S, V, t[1], t[2], t[3])
    elif w in ("bwdsoa64", "bwdsoa32"):
        dt = np.float64 if w == "bwdsoa64" else np.float32
        G, dS, dU, dV, _ = inputs.diff_batch(dt)
        g = dev(*inputs.soa_from_mats(G))
        out = api.ksvd2_batch(*g, plain=True)
        up = dev(*(np.ascontiguousarray(x) for x in (dS[:, 0], dS[:, 1])),
                 *(np.ascontiguousarray(dU[:, i, j]) for j in range(2) for i in range(2)),
                 *(np.ascontiguousarray(dV[:, i, j]) for j in range(2) for i in range(2)))
        for _ in range(reps + 1):
            api.ksvd2_backward_soa(out, up[0], up[1], torch.stack(up[2:6]), torch.stack(up[6:10]))
    elif w in ("cplx128", "cplx64"):
        G = torch.from_numpy(inputs.complex_batch(np.complex128 if w == "cplx128"
                                                  else np.complex64)).cuda()
        for _ in range(reps + 1):
            api.ksvd2c(G)
    elif w == "rect64":
        from paper_2407_13116_amd import sweep as sw

        pr = sw.PackedRect(inputs.rect_batch(), dtype=np.float64)
        for _ in range(reps):
            pr.reset()
            sw.svd_rect_device(pr)
    elif w == "copy":
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(reps):
            dst.copy_(src)
    elif w in ("sweep4", "sweep4rr"):
        from paper_2407_13116_amd import sweep as sw

        p = sw.Packed(inputs.sweep_uniform())
        for _ in range(reps):
            sw.kog_sweep_batch(p, max_sweeps=1, tol_factor=-1.0, mode="persistent",
                               ordering="round-robin" if w == "sweep4rr" else "modulus")
    elif w in ("sweep5", "sweep5f32"):
        from paper_2407_13116_amd import sweep as sw

        dt = np.float64 if w == "sweep5" else np.float32
        p = sw.Packed(inputs.sweep_uneven(dtype=dt), dtype=dt)
        for _ in range(reps):
            sw.kog_sweep_batch(p, max_sweeps=1, tol_factor=-1.0, mode="persistent")
    elif w in ("sgrad64", "sgrad32"):
        from paper_2407_13116_amd import sweep as sw

        dt = np.float64 if w == "sgrad64" else np.float32
        p = sw.Packed(inputs.sweep_uniform() if w == "sgrad64" else inputs.sweep_uneven(dtype=dt),
                      dtype=dt)
        out = sw.kog_sweep_batch(p, max_sweeps=1, tol_factor=-1.0, mode="persistent")
        ds = torch.from_numpy(np.random.default_rng(17).standard_normal(int(p.n.sum()))
                              .astype(dt)).cuda()
        for _ in range(reps + 1):
            sw.sigma_grad(p, out["U"], out["V"], ds, workspace=out["workspace"])
    else:
        print(f"unknown workload {w}; one of:{PROFILE_WORKLOADS}", file=sys.stderr)
        return 2
    torch.cuda.synchronize()
    log(f"[bench] profile workload {w}: done")
    return 0


def main():
    args = parse()
    if args.profile_workload:
        sys.exit(profile_workload(args.profile_workload, args.reps))
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the batched 2x2 "
              "SVD shards by matrix with no communication, and runs on several GPUs are not "
              "implemented.", file=sys.stderr)
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "no GPU"
    log("[bench] FP64 forward, 2^24 matrices")
    launches = []
    f64, g64, h64 = fwd_case(np.float64, args.steps, args.warmup, per_launch=launches)
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
        "roofline": roofline(f64),
    }
    # HIP-event duration of each timed launch of the headline kernel (ms, launch order)
    res["roofline"]["timed_launch_ms"] = [round(x, 5) for x in launches]
    extra = {}
    if not args.no_extra:
        log("[bench] FP32 forward, 2^24 matrices")
        f32, g32, h32 = fwd_case(np.float32, args.steps, args.warmup)
        a32 = ALG_VALU_SLOTS[np.float32] * f32["B"] / (f32["ms_kernel"] * 1e-3) / 1e12
        extra["fwd_f32"] = {"rate": f32["rate"], "ms_per_launch": f32["ms_kernel"],
                            "GBs": f32["GBs"], "hbm_frac": f32["GBs"] / HBM_PEAK_GBS,
                            "alg_T_lane_ops": a32, "alu_frac": a32 / VALU_LANE_PEAK_T}
        fast_err = {}
        for dt, name in ((np.float64, "fwd_fast_f64"), (np.float32, "fwd_fast_f32")):
            log(f"[bench] {name}: the variant without a correctly rounded hypot, 2^24")
            ff, gf, hf = fwd_case(dt, args.steps, args.warmup, fast=True)
            extra[name] = {"rate": ff["rate"], "ms_per_launch": ff["ms_kernel"],
                           "GBs": ff["GBs"], "hbm_frac": ff["GBs"] / HBM_PEAK_GBS}
            fast_err[name] = sigma_error_histogram(gf, hf, hf["labels"], dt)
            del gf, hf
        if not args.no_cpu:
            extra["fwd_fast_f64"]["cpu_baseline"] = oracle_beside("fast")
        for cdt, name in ((np.complex128, "complex_c128"), (np.complex64, "complex_c64")):
            log(f"[bench] {name}: complex 2x2 SVD, 2^22 matrices")
            extra[name] = complex_case(cdt, args.steps, args.warmup)
        if not args.no_cpu:
            extra["complex_c128"]["cpu_baseline"] = oracle_beside("complex")
        for dt, name in ((np.float64, "fwdbwd_f64"), (np.float32, "fwdbwd_f32")):
            log(f"[bench] {name}, 2^22 matrices")
            fb = fwdbwd_case(dt, args.steps, args.warmup)
            # binding bound of the pair: the forward at its algorithmic VALU work, the
            # backward at its algorithmic HBM bytes (it is bound by streaming)
            t_fwd = ALG_VALU_SLOTS[dt] * fb["B"] / (VALU_LANE_PEAK_T * 1e12)
            t_bwd = BYTES_BWD[dt] * fb["B"] / (HBM_PEAK_GBS * 1e9)
            extra[name] = {"rate": fb["rate"], "ms_per_step": fb["ms_kernel"], "GBs": fb["GBs"],
                           "hbm_frac": fb["GBs"] / HBM_PEAK_GBS,
                           "bound_ms": (t_fwd + t_bwd) * 1e3,
                           "frac_of_bound": (t_fwd + t_bwd) * 1e3 / fb["ms_kernel"],
                           "path": "torch.autograd.Function (api.svd2x2) + torch.autograd.grad"}
        from paper_2407_13116_amd import inputs as _inp

        log("[bench] sweep: 256 x (n=256) FP64")
        extra["sweep_uniform_f64"] = sweep_case(_inp.sweep_uniform(), np.float64,
                                                traffic_profile=SWEEP_TRAFFIC_PROFILE)
        for dt, name in ((np.float64, "sweep_uneven_f64"), (np.float32, "sweep_uneven_f32")):
            log(f"[bench] sweep: 1,000 uneven orders, {name}")
            extra[name] = sweep_case(_inp.sweep_uneven(dtype=dt), dt)
        log("[bench] rectangular: 256 x (512 x 256) FP64")
        extra["rect_f64"] = rect_case(np.float64)
        if not args.no_cpu:
            extra["rect_f64"]["cpu_baseline"] = oracle_beside("rect", seconds=5.0)
        log(f"[bench] rect: {extra['rect_f64']}")
        log("[bench] sigma accuracy: the whole 2^24 batches against the double-word reference")
        ref = ("every matrix of the 2^24 batch against a double-word (about 2^-100) "
               "reference of sigma_1, sigma_2 (bench.sigma_ref)")
        extra["max_rel_err_sigma_ulp"] = {
            "f64": sigma_error_histogram(g64, h64, h64["labels"], np.float64),
            "f32": sigma_error_histogram(g32, h32, h32["labels"], np.float32),
            "unit": "eps (2^-53 / 2^-24)", "sample": ref}
        extra["max_rel_err_sigma_ulp_fast"] = dict(fast_err, unit="eps (2^-53 / 2^-24)",
                                                   sample=ref)
    res["extra"] = extra
    if not args.no_cpu:
        log("[bench] oracle CPU baseline")
        res["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
