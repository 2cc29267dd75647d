"""Launch-shape autotuner for the batch kernels.

The persistent batch kernels take one knob, the resident workgroups per
compute unit (each workgroup is one wavefront working on one block at a
time, its block and hash table in LDS).  Fewer workgroups leave latency
uncovered; more raise LDS and register pressure and the tail of the last
round of blocks.  The best value depends on the mix of element classes and
block sizes, so it is measured per batch signature and cached in a JSON
file (``$BSG_TUNE_CACHE``, default ``~/.cache/bsg/tune.json``).
"""
from __future__ import annotations

import json
import math
import os
import statistics

import torch

CANDIDATES = (1, 2, 4, 8, 16, 32)


def cache_path() -> str:
    return os.environ.get("BSG_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "bsg", "tune.json"))


def signature(plan, direction: str) -> str:
    """Device, direction, and the per-class block counts rounded to powers
    of two: batches that differ only in detail share a tuned value."""
    from . import block_elems
    classes: dict[tuple, int] = {}
    for n, e, b in plan.meta:
        nb = block_elems(e, b)
        blocks = n // nb + (1 if (n % nb) // 8 else 0)
        ec = e if e in (1, 2, 4, 8, 12, 16) else 0
        key = (ec, nb * e > 8192)
        classes[key] = classes.get(key, 0) + blocks
    parts = [f"e{k[0]}{'L' if k[1] else 'S'}:{int(round(math.log2(v)))}" for k, v in
             sorted(classes.items()) if v > 0]
    name = torch.cuda.get_device_name(plan.device)
    return f"{name}|{direction}|{','.join(parts)}"


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db: dict) -> None:
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def time_ms(fn, reps: int = 3, warmup: int = 1, stream=None) -> list[float]:
    """Device time of fn() per call (ms), measured with events on the stream."""
    st = stream if stream is not None else torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    out = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        fn()
        b.record(st)
        b.synchronize()
        out.append(a.elapsed_time(b))
    return out


def tune(plan, direction: str, candidates=CANDIDATES, reps: int = 3, use_cache: bool = True):
    """Best waves_per_cu for plan.compress ('compress') or plan.decompress
    ('decompress').  Returns (best, {candidate: median ms})."""
    key = signature(plan, direction)
    db = _load() if use_cache else {}
    if use_cache and key in db:
        return int(db[key]["best"]), {int(k): v for k, v in db[key]["ms"].items()}
    call = plan.compress if direction == "compress" else plan.decompress
    ms = {}
    for w in candidates:
        ms[w] = statistics.median(time_ms(lambda: call(waves_per_cu=w), reps=reps))
    best = min(ms, key=ms.get)
    if use_cache:
        db[key] = {"best": best, "ms": {str(k): v for k, v in ms.items()}}
        _store(db)
    return best, ms
