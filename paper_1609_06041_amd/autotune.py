"""Autotuner for the batched solve's tile shapes and workgroup placement.

Every candidate of ``CANDIDATES`` is set on the batch, the captured loop is
replayed a few times (device time from HIP events, ``ctpd_batch_time_loop``)
and the fastest is kept.  Results are cached in a JSON file keyed by the
device name and the multiset of problem geometries, so a later batch of the
same composition reuses the choice without timing.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from . import ctpd

CANDIDATES = [dict(placement=p, tv_threads=t, fwd_form=f) for p in (0, 1) for t in (1024, 512) for f in (0, 1)]


def signature(geoms, iters: int, tv_iters: int) -> str:
    key = json.dumps({"device": torch.cuda.get_device_name(), "geoms": sorted(map(list, geoms)),
                      "iters": int(iters), "tv_iters": int(tv_iters), "knobs": sorted(CANDIDATES[0])})
    return hashlib.sha1(key.encode()).hexdigest()[:16]


def autotune(batch: ctpd.Batch, bs, ws, betas, iters: int, tv_iters: int = 10, cache_path: str | None = None,
             reps: int = 3) -> dict:
    """Choose and set the batch's tiles.  Returns {"tiles": ..., "timings_ms": [...], "cached": bool}."""
    sig = signature(batch.geoms, iters, tv_iters)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if sig in cache:
        batch.set_tiles(**cache[sig]["tiles"])
        return dict(cache[sig], cached=True)
    batch.lowdose_solve(bs, ws, betas, iters, tv_iters=tv_iters)   # sets the batch up for timing
    timings = []
    for cand in CANDIDATES:
        try:
            batch.set_tiles(**cand)
        except ctpd.CtpdError:   # a choice the batch's geometries do not allow (an image too large for a form)
            timings.append(float("inf"))
            continue
        batch.time_loop(iters, tv_iters, 1)   # capture + warm
        timings.append(batch.time_loop(iters, tv_iters, reps))
    best = CANDIDATES[min(range(len(CANDIDATES)), key=timings.__getitem__)]
    batch.set_tiles(**best)
    entry = {"tiles": best, "timings_ms": [dict(c, ms=t) for c, t in zip(CANDIDATES, timings)]}
    if cache_path:
        cache[sig] = entry
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return dict(entry, cached=False)
