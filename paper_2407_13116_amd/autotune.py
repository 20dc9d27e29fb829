"""Autotuner of the persistent sweep kernels.

For each (dtype, order bucket) present in a batch, time one sweep of a sample
of that bucket's matrices under every candidate workgroup size, keep the
fastest, and install it in the library's tuning table (kog_sweep_tune).
Results are cached in a JSON file keyed by device name, dtype and bucket, so a
later process reuses them without timing again.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import sweep as sw

CANDIDATES = (256, 512, 1024)
CACHE = os.environ.get("KSVD2_TUNE_CACHE",
                       os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json"))
BUCKET_EDGES = (64, 128, 256, 512)


def bucket_of(n: int) -> int:
    for b, e in enumerate(BUCKET_EDGES):
        if n <= e:
            return b
    return len(BUCKET_EDGES)


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(tab):
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def _time_one(mats, dtype, block, bucket, reps=2):
    sw.set_tuning(dtype, bucket, block)
    p = sw.Packed(mats, dtype=np.float64 if dtype == torch.float64 else np.float32)
    G0 = p.G.clone()
    best = float("inf")
    for _ in range(reps):
        p.G.copy_(G0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sw.kog_sweep_batch(p, max_sweeps=1, tol_factor=-1.0, mode="persistent")
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune(mats, dtype=torch.float64, sample: int = 64, force: bool = False, verbose=False):
    """Tune every bucket present in `mats` (list of square numpy matrices)."""
    dev = torch.cuda.get_device_name()
    tab = _load()
    chosen = {}
    by_bucket = {}
    for m in mats:
        by_bucket.setdefault(bucket_of(m.shape[0]), []).append(m)
    for b, ms in sorted(by_bucket.items()):
        key = f"{dev}|{'f64' if dtype == torch.float64 else 'f32'}|{b}"
        if key in tab and not force:
            blk = tab[key]["block"]
        else:
            rng = np.random.default_rng(b)
            pick = [ms[i] for i in rng.choice(len(ms), min(sample, len(ms)), replace=False)]
            times = {blk: _time_one(pick, dtype, blk, b) for blk in CANDIDATES}
            blk = min(times, key=times.get)
            tab[key] = {"block": blk, "ms": times, "sample": len(pick)}
            if verbose:
                print(f"[autotune] {key}: {times} -> {blk}", flush=True)
        sw.set_tuning(dtype, b, blk)
        chosen[b] = blk
    try:
        _save(tab)
    except OSError:
        pass
    return chosen
