"""Named GPU workloads for profiling runs (rocprofv3 --kernel-trace / --pmc).

python -m paper_2407_13116_amd.probe --workload NAME [--reps K]

  fwd64 / fwd32     the 2^24-matrix forward workload (k_fwd_soa)
  fast64 / fast32   the same workload, the variant without a correctly rounded hypot
                    (--fast selects that variant for the cls* workloads too)
  cls15_64 / cls13_64 / cls15_32 / cls13_32
                    2^22 matrices of one class only (general, upper triangular; exponents
                    in [-20,20]): no lane divergence between classes, so the per-wave VALU
                    instruction count is the per-matrix path length of that class
  bwd64 / bwd32     the 2^22-matrix backward (k_bwd)
  cplx128 / cplx64  the 2^22-matrix complex 2x2 SVD (k_fwd_c)
  rect64            256 tall 512 x 256 FP64 matrices: k_qrcp, the sweep, k_qapply
  copy              a plain 1 GiB device-to-device copy (counter calibration: FETCH_SIZE
                    and WRITE_SIZE should each read 1 GiB)
  sweep4            one persistent sweep of the 256 x (n=256) FP64 workload
"""
from __future__ import annotations

import argparse
import sys

import numpy as np
import torch

from . import api, inputs


def _dev(*a):
    return [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in a]


def _fwd(g, reps, fast=False):
    d = _dev(*g)
    out = api.ksvd2_batch(*d, plain=False, fast=fast)
    for _ in range(reps):
        api.ksvd2_batch(*d, plain=False, out=out, fast=fast)


def _class_batch(dtype, tri, B=1 << 22, seed=31):
    rng = np.random.default_rng(seed)
    G = inputs.signed_pow2_entries(rng, (B, 2, 2), -20, 20, dtype)
    if tri:
        G[:, 1, 0] = 0
    return inputs.soa_from_mats(G)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--fast", action="store_true")
    a = ap.parse_args(argv)
    w, reps = a.workload, a.reps
    if w in ("fwd64", "fwd32", "fast64", "fast32"):
        dt = np.float64 if w.endswith("64") else np.float32
        _fwd(inputs.forward_sweep(dt), reps, fast=w.startswith("fast"))
    elif w.startswith("cls"):
        dt = np.float64 if w.endswith("64") else np.float32
        _fwd(_class_batch(dt, tri=w.startswith("cls13")), reps, fast=a.fast)
    elif w in ("bwd64", "bwd32"):
        dt = np.float64 if w == "bwd64" else np.float32
        G, dS, dU, dV, _ = inputs.diff_batch(dt)
        t = _dev(G, dS, dU, dV)
        U, S, V = api.svd2x2_raw(t[0])
        for _ in range(reps):
            api.svd2x2_backward(U, S, V, t[1], t[2], t[3])
    elif w in ("cplx128", "cplx64"):
        G = torch.from_numpy(inputs.complex_batch(np.complex128 if w == "cplx128"
                                                  else np.complex64)).cuda()
        for _ in range(reps + 1):
            api.ksvd2c(G)
    elif w == "rect64":
        from . import sweep as sw

        pr = sw.PackedRect(inputs.rect_batch(), dtype=np.float64)
        for _ in range(reps):
            pr.reset()
            sw.svd_rect_device(pr)
    elif w == "copy":
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(reps):
            dst.copy_(src)
    elif w == "sweep4":
        from . import sweep as sw

        p = sw.Packed(inputs.sweep_uniform())
        for _ in range(reps):
            sw.kog_sweep_batch(p, max_sweeps=1, tol_factor=-1.0, mode="persistent")
    else:
        print(f"unknown workload {w}", file=sys.stderr)
        return 2
    torch.cuda.synchronize()
    print(f"probe {w}: done", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
