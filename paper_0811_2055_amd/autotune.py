"""Schedule autotuner driver: runs lod_autotune on an input and keeps the
winning schedule in a JSON cache keyed by device, problem-size bucket, n and
maximum depth (default path: $LOD_TUNE_CACHE or ~/.cache/lod_tune.json)."""
from __future__ import annotations

import json
import math
import os

from . import lib


def cache_path(path=None):
    return path or os.environ.get("LOD_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache",
                                                                       "lod_tune.json")


def cache_key(N: int, params: lib.BuildParams, device_name: str) -> str:
    bucket = int(math.log2(max(N, 1)))
    return f"{device_name}|N2^{bucket}|n{params.n}|D{params.max_depth}|L{params.density_level}|a{params.alpha}"


def lookup(N: int, params: lib.BuildParams, device_name: str, path=None):
    p = cache_path(path)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        return json.load(f).get(cache_key(N, params, device_name))


def tune(builder: lib.Builder, x, y, z, m, snap_offsets=None, path=None, device_name=None):
    """Tune `builder` in place on this input and record the result."""
    import torch
    dev_name = device_name or torch.cuda.get_device_name(x.device)
    best, table = builder.autotune(x, y, z, m, snap_offsets)
    rec = {"mode": best.mode, "select_threads": best.select_threads,
           "persistent_blocks": best.persistent_blocks,
           "ms": min(t for _, t in table), "candidates": table}
    p = cache_path(path)
    os.makedirs(os.path.dirname(p), exist_ok=True)
    data = {}
    if os.path.exists(p):
        with open(p) as f:
            data = json.load(f)
    data[cache_key(builder.N, builder.params, dev_name)] = rec
    with open(p, "w") as f:
        json.dump(data, f, indent=1)
    return rec


def apply_cached(builder: lib.Builder, device_name: str, path=None) -> bool:
    rec = lookup(builder.N, builder.params, device_name, path)
    if not rec:
        return False
    builder.params.mode = rec["mode"]
    builder.params.select_threads = rec["select_threads"]
    builder.params.persistent_blocks = rec["persistent_blocks"]
    return True
