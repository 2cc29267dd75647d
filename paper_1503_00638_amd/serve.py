"""Request loop with continuous batching over device-resident payloads.

Requests (compress a payload, or decompress its stream) arrive over time.
The loop admits every arrived request whose output (plus, for
compression, its share of the workspace) fits in what is left of the HBM
budget, and gathers the admitted ones into one batch call per direction
(the batch entry points: one persistent kernel per element class walks
every block of every request, blocks and requests being independent units
as in Section 4.2).  A batch is enqueued on one of several streams, so
requests that arrive while others run are admitted as soon as a stream
and memory are free, and their work overlaps on the device.  Completion is
read from device events, so latency runs from the scheduled arrival to the
end of the request's batch on the GPU.

Everything the loop needs on the device is allocated when the server is
built: the budget is one arena (outputs and workspaces of requests in
flight are carved out of it by a first-fit allocator on the host), and
each stream owns its descriptor tables (pinned host + device) and its
result words.  The request loop itself allocates no device or pinned
memory; it builds tables on the host and calls the C-ABI on those buffers.

The plain per-request path (one request per call of the single-stream
entry points, in arrival order on one stream, on the same arena) runs the
same arrivals for comparison.
"""
from __future__ import annotations

import bisect
import collections
import ctypes
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import BSG_SCHED_STRIDED, _lib, compress_bound, workspace_size
from .workloads import POOL_BLOCK_ELEMS

ELEM = 4
ALIGN = 256


@dataclass
class Served:
    rid: int
    op: str
    nbytes: int
    t_arrival: float
    t_admit: float = 0.0
    t_done: float = 0.0  # from the device completion event
    batch: int = -1


class Arena:
    """First-fit allocator over one device buffer, kept on the host: regions
    are (offset, size) pairs aligned to 256 bytes; freed regions coalesce
    with their neighbours."""

    def __init__(self, nbytes: int, device):
        self.nbytes = nbytes - nbytes % ALIGN
        self.buf = torch.empty(max(self.nbytes, ALIGN), dtype=torch.uint8, device=device)
        self.base = self.buf.data_ptr()
        self.starts, self.sizes = [0], [self.nbytes]  # free list, sorted by start
        self.used = 0

    def alloc(self, n: int):
        n = max(ALIGN, -(-n // ALIGN) * ALIGN)
        for k, sz in enumerate(self.sizes):
            if sz >= n:
                off = self.starts[k]
                if sz == n:
                    del self.starts[k], self.sizes[k]
                else:
                    self.starts[k] += n
                    self.sizes[k] -= n
                self.used += n
                return off, n
        return None

    def free(self, region) -> None:
        off, n = region
        k = bisect.bisect_left(self.starts, off)
        self.starts.insert(k, off)
        self.sizes.insert(k, n)
        self.used -= n
        if k + 1 < len(self.starts) and off + n == self.starts[k + 1]:  # merge right
            self.sizes[k] += self.sizes[k + 1]
            del self.starts[k + 1], self.sizes[k + 1]
        if k > 0 and self.starts[k - 1] + self.sizes[k - 1] == off:  # merge left
            self.sizes[k - 1] += self.sizes[k]
            del self.starts[k], self.sizes[k]

    def ptr(self, region) -> int:
        return self.base + region[0]

    def view(self, region, n: int) -> torch.Tensor:
        return self.buf[region[0]:region[0] + n]


class _Slot:
    """What one stream needs for one batch (or one plain request), allocated
    once: descriptor tables for each direction (pinned host + device) and
    the device result words."""

    def __init__(self, device, max_batch: int):
        L = _lib.lib()
        self.stream = torch.cuda.Stream(device)
        self.tb = int(L.bsg_batch_table_bytes(max_batch))
        self.host = {d: torch.empty(self.tb, dtype=torch.uint8, pin_memory=True) for d in "cd"}
        self.dev = {d: torch.empty(self.tb, dtype=torch.uint8, device=device) for d in "cd"}
        self.nbytes = torch.zeros(max_batch, dtype=torch.int64, device=device)
        self.status = torch.zeros(max_batch, dtype=torch.int32, device=device)
        self.rows = (_lib.Chunk * max_batch)()


@dataclass
class _Flight:
    slot: _Slot
    done: object
    reqs: list
    regions: list
    outs: dict = field(default_factory=dict)  # rid -> its output region in the arena


class Server:
    def __init__(self, pool, device="cuda", hbm_budget: int = 64 << 30, n_streams: int = 4,
                 max_batch: int = 64, launch=((0, BSG_SCHED_STRIDED), (0, BSG_SCHED_STRIDED))):
        """launch: (waves_per_cu, schedule) of the batch kernels for
        compression and for decompression (0 = the library default)."""
        self.pool = pool
        self.device = torch.device(device)
        self.budget = hbm_budget
        self.max_batch = max_batch
        self.lc, self.ld = launch
        self.arena = Arena(hbm_budget, self.device)
        self.slots = [_Slot(self.device, max_batch) for _ in range(n_streams)]
        self.ws = {}  # per payload: single-call compression workspace bytes
        for e in pool:
            self.ws[id(e)] = workspace_size(e.n, ELEM, POOL_BLOCK_ELEMS)

    # -- device bytes a request's output (and workspace share) needs --------
    def _out_bytes(self, req) -> int:
        e = self.pool[req.payload]
        if req.op == "compress":
            return compress_bound(e.n, ELEM, POOL_BLOCK_ELEMS)
        return e.nbytes

    def request_bytes(self, req) -> int:
        """Arena bytes a request holds in flight: its output and, for
        compression, its workspace (with room for the batch call's
        per-block prefix sums)."""
        e = self.pool[req.payload]
        extra = 0
        if req.op == "compress":
            blocks = -(-e.n // POOL_BLOCK_ELEMS)
            extra = self.ws[id(e)] + 8 * (blocks + 1 + 1024) + 4 * ALIGN
        return self._out_bytes(req) + extra

    # -- one batch: both directions on one stream ---------------------------
    def _batch_table(self, slot, kind, reqs, outs):
        """Descriptor table for reqs in slot's host buffer of `kind`."""
        L = _lib.lib()
        rows = slot.rows
        for k, r in enumerate(reqs):
            e = self.pool[r.payload]
            o = outs[k]
            if kind == "c":
                rows[k] = _lib.Chunk(e.data.data_ptr(), 0, self.arena.ptr(o), o[1], e.n, ELEM,
                                     POOL_BLOCK_ELEMS)
            else:
                rows[k] = _lib.Chunk(e.stream.data_ptr(), e.stream_len, self.arena.ptr(o), 0, e.n,
                                     ELEM, POOL_BLOCK_ELEMS)
        host = ctypes.c_void_p(slot.host[kind].data_ptr())
        _lib.check(L.bsg_batch_build_table(rows, len(reqs), host, slot.tb), "batch_build_table")
        return host

    def _admit(self, reqs_in, limit):
        """Take requests from the front of reqs_in while their outputs (and
        the batch workspace) fit the arena; returns (taken, regions, outs)."""
        take, regions, outs = [], [], {}
        while reqs_in and len(take) < limit:
            r = reqs_in[0]
            reg = self.arena.alloc(self._out_bytes(r))
            if reg is None:
                break
            reqs_in.popleft()
            take.append(r)
            regions.append(reg)
            outs[r.rid] = reg
        return take, regions, outs

    def _launch_batch(self, slot, take, outs):
        """Enqueue the batch on slot's stream; returns extra arena regions
        (the compression workspace) or None when it does not fit."""
        L = _lib.lib()
        st = slot.stream
        comp = [r for r in take if r.op == "compress"]
        decs = [r for r in take if r.op == "decompress"]
        extra = []
        if comp:
            host = self._batch_table(slot, "c", comp, [outs[r.rid] for r in comp])
            wsb = int(L.bsg_batch_workspace_size(host))
            ws = self.arena.alloc(wsb)
            if ws is None:
                return None
            extra.append(ws)
        with torch.cuda.stream(st):
            if comp:
                slot.dev["c"].copy_(slot.host["c"], non_blocking=True)
                _lib.check(L.bsg_batch_compress(host, ctypes.c_void_p(slot.dev["c"].data_ptr()),
                                                ctypes.c_void_p(slot.nbytes.data_ptr()),
                                                ctypes.c_void_p(self.arena.ptr(ws)), ws[1],
                                                self.lc[0], self.lc[1],
                                                ctypes.c_void_p(st.cuda_stream)),
                           "batch_compress")
            if decs:
                hostd = self._batch_table(slot, "d", decs, [outs[r.rid] for r in decs])
                slot.dev["d"].copy_(slot.host["d"], non_blocking=True)
                slot.status.zero_()
                _lib.check(L.bsg_batch_decompress(hostd, ctypes.c_void_p(slot.dev["d"].data_ptr()),
                                                  ctypes.c_void_p(slot.status.data_ptr()),
                                                  self.ld[0], self.ld[1],
                                                  ctypes.c_void_p(st.cuda_stream)),
                           "batch_decompress")
        return extra

    def _launch_single(self, slot, req, out):
        """One request through the single-stream entry points."""
        L = _lib.lib()
        e = self.pool[req.payload]
        st = ctypes.c_void_p(slot.stream.cuda_stream)
        if req.op == "compress":
            ws = self.arena.alloc(self.ws[id(e)])
            if ws is None:
                return None
            _lib.check(L.bsg_compress_lz4(ctypes.c_void_p(e.data.data_ptr()),
                                          ctypes.c_void_p(self.arena.ptr(out)), e.n, ELEM,
                                          POOL_BLOCK_ELEMS, out[1],
                                          ctypes.c_void_p(slot.nbytes.data_ptr()),
                                          ctypes.c_void_p(self.arena.ptr(ws)), ws[1], st),
                       "compress_lz4")
            return [ws]
        with torch.cuda.stream(slot.stream):
            slot.status[:1].zero_()
        _lib.check(L.bsg_decompress_lz4(ctypes.c_void_p(e.stream.data_ptr()), e.stream_len,
                                        ctypes.c_void_p(self.arena.ptr(out)), e.n, ELEM,
                                        POOL_BLOCK_ELEMS, ctypes.c_void_p(slot.status.data_ptr()),
                                        st), "decompress_lz4")
        return []

    def _collect(self, fl, keep, kept):
        """Copies of the kept requests' results (tests and sampled checks).
        They are made on the batch's own stream, so that the slot's next
        batch cannot overwrite its length and status words first, and they
        are finished before the arena regions are freed: a freed region may
        be handed at once to a batch on another stream."""
        comp = [r for r in fl.reqs if r.op == "compress"]
        decs = [r for r in fl.reqs if r.op == "decompress"]
        copied = False
        with torch.cuda.stream(fl.slot.stream):
            for lst, word in ((comp, fl.slot.nbytes), (decs, fl.slot.status)):
                for k, r in enumerate(lst):
                    if r.rid in keep:
                        reg = fl.outs[r.rid]
                        kept[r.rid] = (self.arena.view(reg, reg[1]).clone(),
                                       word[k:k + 1].clone())
                        copied = True
        if copied:
            fl.slot.stream.synchronize()

    def run(self, requests, mode: str = "batch", keep=()):
        """Serve `requests` (sorted by arrival) in real time.  mode 'batch'
        = continuous batching over the streams; 'single' = the plain
        per-request path on one stream.  Returns (served, kept results,
        number of launches).  Kept results (output bytes, length or status
        word) are copies made when the request completes."""
        reqs = sorted(requests, key=lambda r: r.t_arrival)
        served = {r.rid: Served(r.rid, r.op, r.nbytes, r.t_arrival) for r in reqs}
        keep = set(keep)
        kept = {}
        for r in reqs:
            if self.request_bytes(r) > self.budget:
                raise ValueError(f"request {r.rid} needs {self.request_bytes(r)} bytes, over the "
                                 "budget")
        slots = self.slots if mode == "batch" else self.slots[:1]
        limit = self.max_batch if mode == "batch" else 1
        free = collections.deque(slots)
        inflight: list[_Flight] = []
        pending = collections.deque()
        nxt = done = nbatch = 0
        torch.cuda.synchronize(self.device)
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(slots[0].stream)
        ref.synchronize()
        events = [torch.cuda.Event(enable_timing=True) for _ in range(len(slots) + 1)]
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
                    if keep:
                        self._collect(fl, keep, kept)
                    for reg in fl.regions:
                        self.arena.free(reg)
                    done += len(fl.reqs)
                    inflight.remove(fl)
                    free.append(fl.slot)
                    events.append(fl.done)
                    progressed = True
            while pending and free:
                take, regions, outs = self._admit(pending, limit)
                if not take:
                    break  # the oldest request waits for memory
                slot = free[0]
                extra = (self._launch_batch(slot, take, outs) if mode == "batch"
                         else self._launch_single(slot, take[0], outs[take[0].rid]))
                if extra is None:  # the workspace does not fit: give the requests back
                    for reg in regions:
                        self.arena.free(reg)
                    pending.extendleft(reversed(take))
                    break
                free.popleft()
                t_admit = time.perf_counter() - t0
                ev = events.pop()
                ev.record(slot.stream)
                for r in take:
                    served[r.rid].t_admit = t_admit
                    served[r.rid].batch = nbatch
                inflight.append(_Flight(slot, ev, take, regions + extra, outs))
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
        assert self.arena.used == 0
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
