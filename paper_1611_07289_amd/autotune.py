"""Autotuner for the forward tile shape of a plan.

Every candidate tile shape (tile_w x tile_h pixels per workgroup with the
tile's voxel box staged in LDS, or 0 x 0 for the global-memory walk) is
applied with pvr_plan_set_tiles and the simulation is timed with HIP events; the
fastest shape is kept and remembered in a JSON cache keyed by the workload
signature (problem sizes, patch sizes, stack frames), so later plans of the
same workload skip the search.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Optional, Tuple

import numpy as np

# (0, 0) is the untiled global-memory walk
CANDIDATES = [(0, 0), (16, 16), (32, 8), (8, 32), (64, 4), (16, 8), (8, 16), (8, 8)]
CACHE = os.environ.get("PVR_AUTOTUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "pvr_mi355x",
                                    "autotune.json"))


def signature(plan) -> str:
    h = hashlib.sha1()
    h.update(np.asarray([plan.N, plan.M, plan.V, plan.P], np.int64).tobytes())
    h.update(bytes(plan._g))
    h.update(bytes(plan._s))
    wh = np.asarray([(p.w, p.h) for p in plan._p], np.int32)
    h.update(np.unique(wh, axis=0).tobytes())
    return h.hexdigest()[:16]


def _load_cache(path: str) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(path: str, data: Dict) -> None:
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def tune_tiles(plan, X, y, reps: int = 3, cache: Optional[str] = CACHE,
               candidates=CANDIDATES) -> Tuple[Tuple[int, int], Dict[str, float]]:
    """Pick and apply the fastest forward tile shape for this plan (which must
    be built).  Returns (shape, {shape: ms})."""
    import torch
    key = signature(plan)
    db = _load_cache(cache) if cache else {}
    if key in db:
        tw, th = db[key]["best"]
        plan.set_tiles(tw, th)
        return (tw, th), db[key]["ms"]
    e = torch.empty(plan.N, dtype=torch.float32, device=X.device)
    times = {}
    for tw, th in candidates:
        plan.set_tiles(tw, th)
        plan.simulate(X, y_obs=y, resid=e)  # warm
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        evs[0].record()
        for r in range(reps):
            plan.simulate(X, y_obs=y, resid=e)
            evs[r + 1].record()
        torch.cuda.synchronize()
        ms = sorted(evs[r].elapsed_time(evs[r + 1]) for r in range(reps))[reps // 2]
        times[f"{tw}x{th}"] = ms
    best = min(times, key=times.get)
    tw, th = (int(v) for v in best.split("x"))
    plan.set_tiles(tw, th)
    if cache:
        db[key] = {"best": [tw, th], "ms": times}
        _save_cache(cache, db)
    return (tw, th), times
