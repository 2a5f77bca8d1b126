"""Autotuner of the batched build's schedule.

Every schedule of ``fks_batch_schedules()`` (threads per workgroup x workgroups per CU)
builds the same bytes; they differ only in speed.  ``tune_batch`` times each one on the
caller's batch with HIP events, installs the fastest for the batch's size class
(``fks_batch_set_schedule``: log2 of the map count and of the mean map size) and keeps
the result in a JSON cache keyed by GPU architecture and size class, so later processes
start from the tuned schedule without re-timing.
"""
from __future__ import annotations

import json
import math
import os

from . import fks

CACHE_PATH = os.environ.get("FKS_TUNE_CACHE",
                            os.path.join(os.path.expanduser("~"), ".cache", "fks_mi355x", "schedules.json"))


def size_class(M: int, total_keys: int) -> str:
    lm = int(math.floor(math.log2(max(M, 1))))
    mean = total_keys // max(M, 1)
    ls = int(math.floor(math.log2(max(mean, 1))))
    return f"M2^{lm}/mean2^{ls}"


def _arch() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def load_cache(path: str = CACHE_PATH) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except Exception:
        return {}


def save_cache(data: dict, path: str = CACHE_PATH):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def apply_cached(M: int, total_keys: int, path: str = CACHE_PATH):
    """Install a cached schedule for this size class, if one exists.  Returns it or None."""
    ent = load_cache(path).get(_arch(), {}).get(size_class(M, total_keys))
    if ent:
        fks.fks_batch_set_schedule(M, total_keys, int(ent["schedule"]))
        return int(ent["schedule"])
    return None


def tune_batch(keys, vals, map_offsets, batch_seed: int = 1, reps: int = 3, path: str = CACHE_PATH,
               stream=None) -> dict:
    """Time every schedule on this batch; install and cache the fastest.  Returns
    {"schedule": id, "times_ms": {id: median ms}, "class": size class}."""
    import numpy as np
    import torch
    off = np.asarray(map_offsets, np.uint64)
    M = off.size - 1
    total = int(off[-1])
    s = stream or torch.cuda.current_stream()
    times = {}
    for sched in fks.fks_batch_schedules():
        fks.fks_build_batch_u64(keys, vals, off, batch_seed, schedule=sched, stream=s).destroy()   # warm
        samples = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            b = fks.fks_build_batch_u64(keys, vals, off, batch_seed, schedule=sched, stream=s)
            e1.record(s)
            torch.cuda.synchronize()
            samples.append(e0.elapsed_time(e1))
            b.destroy()
        times[sched] = float(np.median(samples))
    best = min(times, key=times.get)
    fks.fks_batch_set_schedule(M, total, best)
    data = load_cache(path)
    data.setdefault(_arch(), {})[size_class(M, total)] = {"schedule": best, "ms": times[best]}
    save_cache(data, path)
    return {"schedule": best, "times_ms": times, "class": size_class(M, total)}
