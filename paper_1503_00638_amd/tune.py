"""Launch-shape autotuner for the batch kernels.

The persistent batch kernels take two knobs, neither of which changes the
output bytes:

* waves_per_cu, the workgroups per compute unit in the grid (each workgroup
  is one wavefront working on one block at a time, its block and hash
  table in LDS).  Fewer leave latency uncovered; more than LDS lets reside
  at once queue behind the first round, which balances the tail, and at the
  top of the range every workgroup takes only a few blocks (the hardware
  dispatcher then balances the load as for one workgroup per block).
* schedule, how the blocks of an element class are dealt to workgroups:
  every grid-th block (strided) or one contiguous range per workgroup
  (ranges), which walks the chunk table one entry at a time instead of
  searching it per block.

The best pair depends on the mix of element classes, block sizes and chunk
sizes, so it is measured per batch signature and cached in a JSON file
(``$BSG_TUNE_CACHE``, default ``~/.cache/bsg/tune.json``).
"""
from __future__ import annotations

import json
import math
import os
import statistics

import torch

WAVES = (4, 8, 16, 32, 64, 128, 256, 1024, 8192)
SCHEDULES = (0, 1)  # BSG_SCHED_STRIDED, BSG_SCHED_RANGES
CANDIDATES = tuple((w, s) for s in SCHEDULES for w in WAVES)


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
    """Best launch shape (waves_per_cu, schedule) for plan.compress
    ('compress') or plan.decompress ('decompress').  Returns
    (best, {"w,s": median ms})."""
    key = signature(plan, direction)
    db = _load() if use_cache else {}
    if use_cache and key in db and isinstance(db[key].get("best"), list):
        return tuple(db[key]["best"]), dict(db[key]["ms"])
    call = plan.compress if direction == "compress" else plan.decompress
    ms = {}
    for w, s in candidates:
        ms[f"{w},{s}"] = statistics.median(
            time_ms(lambda: call(waves_per_cu=w, schedule=s), reps=reps))
    best = min(candidates, key=lambda c: ms[f"{c[0]},{c[1]}"])
    if use_cache:
        db[key] = {"best": list(best), "ms": ms}
        _store(db)
    return best, ms
