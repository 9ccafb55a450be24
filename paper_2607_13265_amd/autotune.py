"""Autotuner for the batched launch: picks the chunk size (paths in flight per launch sequence)
that minimises render + backward time (the median of several timed steps after a warm-up) for a
given scene / views / depth, and caches the choice in a JSON file keyed by a digest of the
workload."""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np
import torch

from .core import Plan

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")
CANDIDATES = (1 << 21, 1 << 22, 1 << 23, 1 << 24, 1 << 25, 1 << 26, 1 << 27)
MEM_FRACTION = 0.6  # a candidate's render + backward workspaces must fit in this share of free memory


def workload_key(blob: bytes, views, max_depth: int, flags: int, device_name: str) -> str:
    h = hashlib.sha256()
    h.update(blob)
    h.update(np.ascontiguousarray(views).tobytes())
    h.update(f"{max_depth}/{flags}/{device_name}".encode())
    return h.hexdigest()[:24]


def _time_step(plan, params, d, want, reps):
    """Median over reps timed render + backward steps, after one untimed step."""
    out = torch.empty(plan.image_numel, dtype=torch.float32, device=params[0].device)
    grads = [torch.empty_like(p) if w else None for p, w in zip(params, want)]
    ws0, ws1 = plan.workspace(0), plan.workspace(1)
    plan.render(params, 1, out=out, ws=ws0)
    plan.backward(params, 1, d, grads=grads, ws=ws1)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.render(params, 1, out=out, ws=ws0)
        plan.backward(params, 1, d, grads=grads, ws=ws1)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    return float(np.median(ms))


def tune(scene, blob: bytes, views, max_depth: int, params, want=None, flags: int = 0, candidates=CANDIDATES,
         reps: int = 3, cache_path: str = DEFAULT_CACHE, force: bool = False, log=None):
    """Returns (chunk_paths, {candidate: ms}) and records the choice in the cache file."""
    dev_name = torch.cuda.get_device_name(params[0].device)
    key = workload_key(blob, views, max_depth, flags, dev_name)
    cache = {}
    if os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if key in cache and not force:
        return int(cache[key]["chunk_paths"]), cache[key]["timings_ms"]
    want = [True] * len(params) if want is None else want
    total = int(np.sum(np.asarray(views["crop_w"], np.int64) * views["crop_h"] * views["spp"]))
    timings = {}
    for q in candidates:
        if timings and max(timings) >= total:
            break  # a previous candidate already held every path in one chunk
        plan = Plan(scene, views, max_depth, flags, chunk_paths=q)
        plan.set_stats(False)
        free, _ = torch.cuda.mem_get_info(params[0].device)
        if timings and plan.workspace_bytes(0) + plan.workspace_bytes(1) > MEM_FRACTION * free:
            del plan
            break  # larger chunks need more memory still
        d = torch.randn(plan.image_numel, device=params[0].device)
        t0 = time.perf_counter()
        timings[int(q)] = _time_step(plan, params, d, want, reps)
        if log:
            log(f"[autotune] chunk {q}: {timings[int(q)]:.2f} ms ({time.perf_counter() - t0:.1f} s)")
        del plan
        torch.cuda.empty_cache()
    best = min(timings, key=timings.get)
    cache[key] = {"chunk_paths": best, "timings_ms": timings, "views": int(len(views)), "max_depth": int(max_depth),
                  "device": dev_name}
    try:
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    except OSError:
        pass
    return best, timings
