"""Request loop with continuous batching over device-resident payloads.

Requests (compress a payload, or decompress its stream) arrive over time.
The loop admits every arrived request whose memory (input + output +
workspace) fits the remaining HBM budget, and gathers the admitted ones
into one batch call per direction (the batch entry points: one persistent
kernel per element class walks every block of every request, blocks and
requests being independent units as in Section 4.2).  A batch is enqueued
on one of several streams, so requests that arrive while others run are
admitted as soon as a stream and memory are free and their work overlaps on
the device.  Completion is read from device events, so latency runs from
the scheduled arrival to the end of the request's batch on the GPU.

The plain per-request path (one request per call of the single-stream
entry points, in arrival order on one stream) runs the same arrivals for
comparison.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import BatchPlan, compress, compress_bound, decompress, workspace_size
from .workloads import POOL_BLOCK_ELEMS

ELEM = 4


@dataclass
class Served:
    rid: int
    op: str
    nbytes: int
    t_arrival: float
    t_admit: float = 0.0
    t_done: float = 0.0  # from the device completion event
    batch: int = -1
    out: torch.Tensor | None = None  # kept only when asked for
    out_len: torch.Tensor | None = None


@dataclass
class _Flight:
    stream: object
    done: object
    reqs: list
    mem: int
    keep: list = field(default_factory=list)


def request_bytes(req, pool) -> int:
    """Device bytes a request holds while in flight: input + output
    (+ compression workspace)."""
    e = pool[req.payload]
    if req.op == "compress":
        n = e.n
        return e.nbytes + compress_bound(n, ELEM, POOL_BLOCK_ELEMS) + \
            workspace_size(n, ELEM, POOL_BLOCK_ELEMS)
    return e.stream_len + e.nbytes


class Server:
    def __init__(self, pool, device="cuda", hbm_budget: int = 64 << 30, n_streams: int = 4,
                 max_batch: int = 64, waves_per_cu=(0, 0)):
        self.pool = pool
        self.device = torch.device(device)
        self.budget = hbm_budget
        self.streams = [torch.cuda.Stream(self.device) for _ in range(n_streams)]
        self.max_batch = max_batch
        self.wc, self.wd = waves_per_cu

    # -- one batch: both directions on one stream ---------------------------
    def _launch_batch(self, reqs, stream, keep_ids):
        pool = self.pool
        comp = [r for r in reqs if r.op == "compress"]
        decs = [r for r in reqs if r.op == "decompress"]
        keep = []
        with torch.cuda.stream(stream):
            if comp:
                pc = BatchPlan.for_compress([pool[r.payload].data for r in comp], ELEM,
                                            POOL_BLOCK_ELEMS, stream=stream)
                pc.compress(self.wc, stream=stream)
                keep.append(pc)
                for k, r in enumerate(comp):
                    if r.rid in keep_ids:
                        keep_ids[r.rid] = (pc.outs[k], pc.nbytes[k:k + 1])
            if decs:
                pd = BatchPlan.for_decompress([pool[r.payload].stream for r in decs],
                                              [pool[r.payload].stream_len for r in decs],
                                              [pool[r.payload].n for r in decs], ELEM,
                                              POOL_BLOCK_ELEMS, stream=stream)
                pd.decompress(self.wd, stream=stream)
                keep.append(pd)
                for k, r in enumerate(decs):
                    if r.rid in keep_ids:
                        keep_ids[r.rid] = (pd.outs[k], pd.status[k:k + 1])
        return keep

    def _launch_single(self, req, stream, keep_ids):
        e = self.pool[req.payload]
        with torch.cuda.stream(stream):
            if req.op == "compress":
                out, nb = compress(e.data, ELEM, POOL_BLOCK_ELEMS, stream=stream)
                res = (out, nb)
            else:
                out, st = decompress(e.stream, e.stream_len, e.n, ELEM, POOL_BLOCK_ELEMS,
                                     stream=stream)
                res = (out, st)
        if req.rid in keep_ids:
            keep_ids[req.rid] = res
        return [res]

    def run(self, requests, mode: str = "batch", keep=()):
        """Serve `requests` (sorted by arrival) in real time.  mode 'batch'
        = continuous batching over the streams; 'single' = the plain
        per-request path on one stream.  Returns (served, kept outputs)."""
        reqs = sorted(requests, key=lambda r: r.t_arrival)
        served = {r.rid: Served(r.rid, r.op, r.nbytes, r.t_arrival) for r in reqs}
        keep_ids = {rid: None for rid in keep}
        mem = {r.rid: request_bytes(r, self.pool) for r in reqs}
        for r in reqs:
            if mem[r.rid] > self.budget:
                raise ValueError(f"request {r.rid} needs {mem[r.rid]} bytes, over the budget")
        streams = self.streams if mode == "batch" else self.streams[:1]
        free = collections.deque(streams)
        inflight: list[_Flight] = []
        pending = collections.deque()
        used = 0
        nxt = 0
        done = 0
        nbatch = 0
        torch.cuda.synchronize(self.device)
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(streams[0])
        ref.synchronize()
        t0 = time.perf_counter()
        while done < len(reqs):
            now = time.perf_counter() - t0
            while nxt < len(reqs) and reqs[nxt].t_arrival <= now:
                pending.append(reqs[nxt])
                nxt += 1
            progressed = False
            for fl in list(inflight):
                if fl.done.query():
                    t_gpu = ref.elapsed_time(fl.done) * 1e-3
                    for r in fl.reqs:
                        served[r.rid].t_done = t_gpu
                    used -= fl.mem
                    done += len(fl.reqs)
                    inflight.remove(fl)
                    free.append(fl.stream)
                    progressed = True
            while pending and free:
                take, need = [], 0
                limit = self.max_batch if mode == "batch" else 1
                while pending and len(take) < limit and used + need + mem[pending[0].rid] <= self.budget:
                    r = pending.popleft()
                    take.append(r)
                    need += mem[r.rid]
                if not take:
                    break  # the oldest request waits for memory
                st = free.popleft()
                t_admit = time.perf_counter() - t0
                if mode == "batch":
                    held = self._launch_batch(take, st, keep_ids)
                else:
                    held = self._launch_single(take[0], st, keep_ids)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(st)
                for r in take:
                    served[r.rid].t_admit = t_admit
                    served[r.rid].batch = nbatch
                inflight.append(_Flight(st, ev, take, need, held))
                used += need
                nbatch += 1
                progressed = True
            if not progressed:
                if nxt < len(reqs) and not inflight and not pending:
                    wait = reqs[nxt].t_arrival - (time.perf_counter() - t0)
                    if wait > 2e-4:
                        time.sleep(wait - 1e-4)
                else:
                    time.sleep(2e-5)
        torch.cuda.synchronize(self.device)
        kept = {rid: v for rid, v in keep_ids.items() if v is not None}
        return [served[r.rid] for r in reqs], kept, nbatch


def summarize(served, nbatch: int) -> dict:
    lat = np.array([s.t_done - s.t_arrival for s in served]) * 1e3
    U = sum(s.nbytes for s in served)
    t_first = min(s.t_arrival for s in served)
    t_last = max(s.t_done for s in served)
    out = {"requests": len(served), "batches": nbatch,
           "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                          "p99": round(float(np.percentile(lat, 99)), 3),
                          "mean": round(float(lat.mean()), 3),
                          "max": round(float(lat.max()), 3)},
           "sustained_GBps": round(U / (t_last - t_first) / 1e9, 2),
           "offered_GBps": round(U / (max(s.t_arrival for s in served) - t_first) / 1e9, 2),
           "uncompressed_bytes": U}
    for op in ("compress", "decompress"):
        ls = np.array([s.t_done - s.t_arrival for s in served if s.op == op]) * 1e3
        if ls.size:
            out[f"{op}_latency_ms"] = {"p50": round(float(np.percentile(ls, 50)), 3),
                                       "p99": round(float(np.percentile(ls, 99)), 3)}
    return out
