"""Autotuner of the persistent sweep kernels.

For each (dtype, order bucket) present in a batch, time one sweep of a sample of
that bucket's matrices (up to 512: a workgroup per matrix, so a sample that keeps the
256 compute units busy, as the whole batch does; smaller samples favoured wider
workgroups) and search the schedule knobs of the library's tuning table
one after the other (coordinate descent from the defaults): the workgroup size
(waves per matrix), two steps of G per pass or one, the in-place form of that pass
or the second buffer, the number of steps whose U/V rotations are applied together
(the chunk) and a cap on the LDS of the U/V tile.  No setting changes a bit of
the results (every one performs the same operations in the same order), so the
fastest is kept and installed (kog_sweep_set_tuning).  Results are cached in a JSON
file keyed by device name, dtype and bucket, so a later process reuses them without
timing again.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import sweep as sw

# knob -> candidates, searched in this order (the first candidate list is the
# workgroup size: 4, 8 or 16 waves per matrix)
SEARCH = (("block", (256, 512, 1024)),
          ("two", (1, 0)),
          ("inplace", (1, 0)),
          ("chunk", (128, 64, 32, 16)),
          ("rows", (0, 64, 32, 16)))
# the library's defaults (binary64 takes 512 lanes for orders 257-512, binary32 1,024)
DEFAULTS = {"block": {"f64": (256, 512, 512, 512, 1024), "f32": (256, 512, 512, 1024, 1024)},
            "chunk": 128, "two": 1, "inplace": 1,
            "rows": 0}
CANDIDATES = SEARCH[0][1]
CACHE = os.environ.get("KSVD2_TUNE_CACHE",
                       os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json"))
BUCKET_EDGES = (64, 128, 256, 512)
_VERSION = 4   # cache entries of other versions are re-tuned


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


def _default(bucket, dtype):
    d = {k: v for k, v in DEFAULTS.items() if k != "block"}
    d["block"] = DEFAULTS["block"]["f64" if dtype == torch.float64 else "f32"][bucket]
    return d


def _time_setting(p, G0, dtype, bucket, setting, ordering, reps=2):
    sw.set_tuning(dtype, bucket, **setting)
    best = float("inf")
    ws = None
    for _ in range(reps):
        p.G.copy_(G0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        out = sw.kog_sweep_batch(p, max_sweeps=1, tol_factor=-1.0, mode="persistent",
                                 workspace=ws, ordering=ordering)
        e1.record()
        torch.cuda.synchronize()
        ws = out["workspace"]
        best = min(best, e0.elapsed_time(e1))
    return best


def _search(mats, dtype, bucket, ordering):
    """Coordinate descent over SEARCH from the defaults; returns (setting, times)."""
    p = sw.Packed(mats, dtype=np.float64 if dtype == torch.float64 else np.float32)
    G0 = p.G.clone()
    cur = _default(bucket, dtype)
    times = {}
    t_cur = _time_setting(p, G0, dtype, bucket, cur, ordering)
    times[json.dumps(cur, sort_keys=True)] = t_cur
    for knob, cands in SEARCH:
        for v in cands:
            if v == cur[knob]:
                continue
            trial = dict(cur, **{knob: v})
            key = json.dumps(trial, sort_keys=True)
            if key not in times:
                times[key] = _time_setting(p, G0, dtype, bucket, trial, ordering)
            if times[key] < t_cur:
                cur, t_cur = trial, times[key]
    del p, G0
    return cur, t_cur, times


def tune(mats, dtype=torch.float64, sample: int = 512, force: bool = False, verbose=False,
         ordering="modulus"):
    """Tune every bucket present in `mats` (list of square numpy matrices); returns
    {bucket: setting} with the knobs installed."""
    dev = torch.cuda.get_device_name()
    tab = _load()
    chosen = {}
    by_bucket = {}
    for m in mats:
        by_bucket.setdefault(bucket_of(m.shape[0]), []).append(m)
    for b, ms in sorted(by_bucket.items()):
        key = f"{dev}|{'f64' if dtype == torch.float64 else 'f32'}|{b}|{ordering}"
        ent = tab.get(key)
        if ent is not None and ent.get("version") == _VERSION and not force:
            setting = ent["setting"]
        else:
            rng = np.random.default_rng(b)
            pick = [ms[i] for i in rng.choice(len(ms), min(sample, len(ms)), replace=False)]
            setting, t_best, times = _search(pick, dtype, b, ordering)
            tab[key] = {"version": _VERSION, "setting": setting, "ms": t_best,
                        "ms_default": times[json.dumps(_default(b, dtype), sort_keys=True)],
                        "tried": len(times), "sample": len(pick)}
            if verbose:
                print(f"[autotune] {key}: {setting} {t_best:.3f} ms "
                      f"(defaults {tab[key]['ms_default']:.3f} ms)", flush=True)
        sw.set_tuning(dtype, b, **setting)
        chosen[b] = dict(setting)
    try:
        _save(tab)
    except OSError:
        pass
    return chosen
