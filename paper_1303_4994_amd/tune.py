"""Autotuner for batched launches.

Chooses the launch geometry of the persistent batch kernels -- waves per
workgroup, persistent workgroups per compute unit, tiles taken per work-queue
ticket -- by timing candidates on the caller's batch with HIP events.  No
candidate changes any output byte (the geometry only decides which
workgroup encodes which tile).  Results are cached in a JSON file keyed by
the device name and a signature of the batch (dtype mix, ndim, block-size
classes, total size bucket); set APAX_TUNE_CACHE to choose the file.
"""
from __future__ import annotations

import json
import math
import os
import sys

import torch

from . import apax as A

CANDIDATES = [{"waves_per_wg": w, "wgs_per_cu": c, "tiles_per_ticket": t}
              for w in (2, 4, 8) for c in (4, 8, 16) for t in (1, 4)]
DEFAULT = {"waves_per_wg": 4, "wgs_per_cu": 8, "tiles_per_ticket": 4}


def cache_path() -> str:
    return os.environ.get("APAX_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "apax_tune.json"))


def signature(op: int, arrays) -> str:
    """arrays: [(tensor, params), ...] (encode) or [(buf, n, hdr), ...] (decode)."""
    dts, modes, total = {}, {}, 0
    for a in arrays:
        if op == A.OP_ENCODE:
            x, p = a
            dts[str(x.dtype)] = dts.get(str(x.dtype), 0) + 1
            modes[p.get("mode", "lossless")] = 1
            total += x.numel() * x.element_size()
        else:
            info = A.apax_stream_info(a[2])
            dts[str(info["dtype"])] = dts.get(str(info["dtype"]), 0) + 1
            modes[info["mode"]] = 1
            total += int(a[1])
    n = len(arrays)
    mix = ",".join(f"{k}:{round(v / max(1, n), 1)}" for k, v in sorted(dts.items()))
    return f"op{op}|n{2 ** int(math.log2(max(1, n)))}|{mix}|{','.join(sorted(modes))}|" \
           f"GB{2 ** int(math.log2(max(1, total >> 20)))}"


def _device() -> str:
    return torch.cuda.get_device_name(0).replace(" ", "_")


def load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(c: dict):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_batch(b: "A.Batch", reps: int = 3) -> float:
    s = torch.cuda.current_stream()
    b.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        b.run()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(op: int, arrays, candidates=None, reps: int = 3, use_cache: bool = True,
         verbose: bool = False) -> dict:
    """Best geometry for this batch (cached)."""
    key = f"{_device()}|{signature(op, arrays)}"
    cache = load_cache() if use_cache else {}
    if key in cache:
        return cache[key]["tune"]
    best, best_ms, log = None, float("inf"), []
    for cand in candidates or CANDIDATES:
        b = A.Batch.encode(arrays, tune=cand) if op == A.OP_ENCODE else A.Batch.decode(arrays, tune=cand)
        ms = time_batch(b, reps)
        b.close()
        log.append((cand, ms))
        if verbose:
            print(f"tune {cand} {ms:.3f} ms", file=sys.stderr, flush=True)
        if ms < best_ms:
            best, best_ms = cand, ms
    cache[key] = {"tune": best, "ms": best_ms}
    if use_cache:
        save_cache(cache)
    return best
