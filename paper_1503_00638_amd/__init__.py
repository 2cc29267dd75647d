"""MI355X (gfx950) implementation of the radio-data compression scheme of
Masui et al., arXiv:1503.00638: noise-relative rounding (Section 3) and
Bitshuffle, the blocked bit transpose plus per-block LZ4 (Section 4.2).

The compute is the HIP library libbsg.so behind the C-ABI in include/bsg.h;
this module only marshals torch device tensors (device memory and streams)
into those calls.  Every function enqueues on the current torch stream (or
the one given) and returns without synchronising, except the *_sync helpers.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (BSG_ECAPACITY, BSG_ECORRUPT, BSG_EHIP, BSG_EINVAL, BSG_FILTER_BIT,
                   BSG_FILTER_BYTE, BSG_OK, BSG_SCHED_RANGES, BSG_SCHED_STRIDED, BsgError,
                   Header)

__all__ = [
    "round_to_noise", "round_to_noise_i32", "noise_compensation", "round_to_noise_scaled",
    "fullcov_inverse_diag", "round_to_noise_fullcov", "bitshuffle", "bitunshuffle", "compress_bound", "workspace_size",
    "compress", "round_compress", "decompress", "block_elems", "read_header", "BsgError",
    "compress_sync", "decompress_sync", "BSG_OK", "BSG_EINVAL", "BSG_ECAPACITY",
    "BSG_ECORRUPT", "BSG_EHIP", "load", "BatchPlan", "byteshuffle", "byteunshuffle",
    "BSG_FILTER_BIT", "BSG_FILTER_BYTE", "compress_noalloc", "NOALLOC_SCRATCH_BYTES",
    "BSG_SCHED_STRIDED", "BSG_SCHED_RANGES",
]

NOALLOC_SCRATCH_BYTES = _lib.NOALLOC_SCRATCH_BYTES


def load():
    """Load libbsg.so (raises ImportError when it is not built)."""
    return _lib.lib()


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _require_device(*ts):
    for t in ts:
        if t is not None:
            if not t.is_cuda:
                raise ValueError("bsg operates on device tensors only")
            if not t.is_contiguous():
                raise ValueError("bsg needs contiguous tensors")


def _nbytes(t: torch.Tensor) -> int:
    return t.numel() * t.element_size()


def _check_out(out: torch.Tensor, nbytes: int, what: str) -> None:
    """A caller-supplied output must hold the bytes the call writes (the C-ABI
    takes raw pointers and cannot check)."""
    if _nbytes(out) < nbytes:
        raise ValueError(f"{what}: output holds {_nbytes(out)} bytes, the call writes {nbytes}")


def _check_word(t: torch.Tensor, dtype, what: str) -> None:
    """Device result words (stream length, decode status) the kernels write."""
    if t.dtype != dtype or t.numel() < 1:
        raise ValueError(f"{what} must be a {dtype} tensor of at least one element")


def _check_prod_map(prod_map: torch.Tensor | None, P: int, I: int) -> None:
    """prod_map must be int32 (P, 2) with every entry in [0, I): the kernels
    index the autos with it and do not check it."""
    if prod_map is None:
        return
    if prod_map.dtype != torch.int32 or tuple(prod_map.shape) != (P, 2):
        raise ValueError("prod_map must be int32 (P, 2)")
    if prod_map.numel():
        lo, hi = torch.aminmax(prod_map)
        if int(lo.item()) < 0 or int(hi.item()) >= I:
            raise ValueError(f"prod_map entries must lie in [0, {I})")


def block_elems(elem_size: int, block_size: int = 0) -> int:
    r = _lib.lib().bsg_block_elems(elem_size, block_size)
    if r < 0:
        raise BsgError(int(r), "block_elems")
    return int(r)


def round_to_noise(vis: torch.Tensor, autos: torch.Tensor, n_samples: float, f: float,
                   out: torch.Tensor | None = None, prod_map: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
    """vis complex64 (F, P, T), autos float32 (F, I, T) -> rounded vis
    (out may be vis itself for in-place rounding)."""
    _require_device(vis, autos, out, prod_map)
    if vis.dtype != torch.complex64 or autos.dtype != torch.float32:
        raise TypeError("vis must be complex64 and autos float32")
    F, I, T = autos.shape
    if tuple(vis.shape) != (F, I * (I + 1) // 2, T):
        raise ValueError(f"vis {tuple(vis.shape)} does not match autos {tuple(autos.shape)}")
    if out is None:
        out = torch.empty_like(vis)
    _check_out(out, _nbytes(vis), "vis_out")
    _check_prod_map(prod_map, vis.shape[1], I)
    _lib.check(_lib.lib().bsg_round_to_noise(_ptr(vis), _ptr(out), _ptr(autos), F, I, T,
                                              _ptr(prod_map), float(n_samples), float(f),
                                              _stream_ptr(stream)), "round_to_noise")
    return out


def _vis_autos(vis, autos):
    if vis.dtype != torch.complex64 or autos.dtype != torch.float32:
        raise TypeError("vis must be complex64 and autos float32")
    F, I, T = autos.shape
    if tuple(vis.shape) != (F, I * (I + 1) // 2, T):
        raise ValueError(f"vis {tuple(vis.shape)} does not match autos {tuple(autos.shape)}")
    return F, I, T


def noise_compensation(vis: torch.Tensor, autos: torch.Tensor, prod_map: torch.Tensor | None = None,
                       out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Per-(frequency, time) factor on f (float64 (F, T)) that compensates
    the diagonal noise model (Section 3.2)."""
    _require_device(vis, autos, prod_map, out)
    F, I, T = _vis_autos(vis, autos)
    _check_prod_map(prod_map, vis.shape[1], I)
    if out is None:
        out = torch.empty((F, T), dtype=torch.float64, device=vis.device)
    _check_out(out, 8 * F * T, "scale")
    _lib.check(_lib.lib().bsg_noise_compensation(_ptr(vis), _ptr(autos), F, I, T, _ptr(prod_map),
                                                  _ptr(out), _stream_ptr(stream)),
               "noise_compensation")
    return out


def round_to_noise_scaled(vis: torch.Tensor, autos: torch.Tensor, n_samples: float, f: float,
                          scale: torch.Tensor, out: torch.Tensor | None = None,
                          prod_map: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """round_to_noise with G2 multiplied by scale[f][t] (float64 (F, T))."""
    _require_device(vis, autos, scale, out, prod_map)
    F, I, T = _vis_autos(vis, autos)
    if scale.dtype != torch.float64 or tuple(scale.shape) != (F, T):
        raise ValueError("scale must be float64 (F, T)")
    _check_prod_map(prod_map, vis.shape[1], I)
    if out is None:
        out = torch.empty_like(vis)
    _check_out(out, _nbytes(vis), "vis_out")
    _lib.check(_lib.lib().bsg_round_to_noise_scaled(_ptr(vis), _ptr(out), _ptr(autos), F, I, T,
                                                     _ptr(prod_map), float(n_samples), float(f),
                                                     _ptr(scale), _stream_ptr(stream)),
               "round_to_noise_scaled")
    return out


def fullcov_inverse_diag(vis: torch.Tensor, autos: torch.Tensor, out: torch.Tensor | None = None,
                         stream=None) -> torch.Tensor:
    """(Q^-1)_kk per sample and degree of freedom (float64 (F, T, I^2)),
    Q = 2N C of Eqs. rad_full1-3 (I <= 11)."""
    _require_device(vis, autos, out)
    F, I, T = _vis_autos(vis, autos)
    if out is None:
        out = torch.empty((F, T, I * I), dtype=torch.float64, device=vis.device)
    _check_out(out, 8 * F * T * I * I, "qdiag")
    _lib.check(_lib.lib().bsg_fullcov_inverse_diag(_ptr(vis), _ptr(autos), F, I, T, _ptr(out),
                                                    _stream_ptr(stream)), "fullcov_inverse_diag")
    return out


def round_to_noise_fullcov(vis: torch.Tensor, autos: torch.Tensor, n_samples: float, f: float,
                           out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Rounding with the full-covariance noise of each degree of freedom."""
    _require_device(vis, autos, out)
    F, I, T = _vis_autos(vis, autos)
    if out is None:
        out = torch.empty_like(vis)
    _check_out(out, _nbytes(vis), "vis_out")
    _lib.check(_lib.lib().bsg_round_to_noise_fullcov(_ptr(vis), _ptr(out), _ptr(autos), F, I, T,
                                                      float(n_samples), float(f),
                                                      _stream_ptr(stream)),
               "round_to_noise_fullcov")
    return out


def round_to_noise_i32(vis: torch.Tensor, autos: torch.Tensor, n_samples: float, f: float,
                       out: torch.Tensor | None = None, prod_map: torch.Tensor | None = None,
                       stream=None) -> torch.Tensor:
    """Integer visibilities: vis int32 (F, P, T, 2), autos int32 (F, I, T) ->
    rounded vis (out may be vis itself)."""
    _require_device(vis, autos, out, prod_map)
    if vis.dtype != torch.int32 or autos.dtype != torch.int32:
        raise TypeError("vis and autos must be int32")
    F, I, T = autos.shape
    if tuple(vis.shape) != (F, I * (I + 1) // 2, T, 2):
        raise ValueError(f"vis {tuple(vis.shape)} does not match autos {tuple(autos.shape)}")
    if out is None:
        out = torch.empty_like(vis)
    _check_out(out, _nbytes(vis), "vis_out")
    _check_prod_map(prod_map, vis.shape[1], I)
    _lib.check(_lib.lib().bsg_round_to_noise_i32(_ptr(vis), _ptr(out), _ptr(autos), F, I, T,
                                                  _ptr(prod_map), float(n_samples), float(f),
                                                  _stream_ptr(stream)), "round_to_noise_i32")
    return out


def _transpose(fn, x, elem_size, block_size, out, stream, what):
    _require_device(x, out)
    nb = _nbytes(x)
    if nb % elem_size:
        raise ValueError("buffer is not a whole number of elements")
    if out is None:
        out = torch.empty(nb, dtype=torch.uint8, device=x.device)
    if _nbytes(out) < nb:
        raise ValueError("output too small")
    _lib.check(fn(_ptr(x), _ptr(out), nb // elem_size, elem_size, block_size, _stream_ptr(stream)),
               what)
    return out


def bitshuffle(x: torch.Tensor, elem_size: int, block_size: int = 0,
               out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    return _transpose(_lib.lib().bsg_bitshuffle, x, elem_size, block_size, out, stream,
                      "bitshuffle")


def bitunshuffle(x: torch.Tensor, elem_size: int, block_size: int = 0,
                 out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    return _transpose(_lib.lib().bsg_bitunshuffle, x, elem_size, block_size, out, stream,
                      "bitunshuffle")


def byteshuffle(x: torch.Tensor, elem_size: int, block_size: int = 0,
                out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Blosc-style byte shuffle within blocks (the comparison filter)."""
    return _transpose(_lib.lib().bsg_byteshuffle, x, elem_size, block_size, out, stream,
                      "byteshuffle")


def byteunshuffle(x: torch.Tensor, elem_size: int, block_size: int = 0,
                  out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    return _transpose(_lib.lib().bsg_byteunshuffle, x, elem_size, block_size, out, stream,
                      "byteunshuffle")


def compress_bound(n: int, elem_size: int, block_size: int = 0) -> int:
    r = _lib.lib().bsg_compress_bound(n, elem_size, block_size)
    if r < 0:
        raise BsgError(int(r), "compress_bound")
    return int(r)


def workspace_size(n: int, elem_size: int, block_size: int = 0) -> int:
    r = _lib.lib().bsg_compress_workspace_size(n, elem_size, block_size)
    if r < 0:
        raise BsgError(int(r), "workspace_size")
    return int(r)


def _alloc_ws(n, elem_size, block_size, device, workspace):
    need = workspace_size(n, elem_size, block_size)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=device)
    return workspace


def compress(x: torch.Tensor, elem_size: int, block_size: int = 0,
             out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
             nbytes: torch.Tensor | None = None, stream=None, filter: int = BSG_FILTER_BIT):
    """Enqueue compression of x.  Returns (out, nbytes): out is a uint8 buffer
    of compress_bound bytes (or the one given), nbytes a device int64 holding
    the stream length (or BSG_ECAPACITY) once the stream has run."""
    _require_device(x, out, workspace, nbytes)
    total = _nbytes(x)
    if total % elem_size:
        raise ValueError("buffer is not a whole number of elements")
    n = total // elem_size
    if out is None:
        out = torch.empty(compress_bound(n, elem_size, block_size), dtype=torch.uint8,
                          device=x.device)
    workspace = _alloc_ws(n, elem_size, block_size, x.device, workspace)
    if nbytes is None:
        nbytes = torch.empty(1, dtype=torch.int64, device=x.device)
    _check_word(nbytes, torch.int64, "nbytes")
    _lib.check(_lib.lib().bsg_compress_lz4_filter(_ptr(x), _ptr(out), n, elem_size, block_size,
                                                   int(filter), _nbytes(out), _ptr(nbytes),
                                                   _ptr(workspace), _nbytes(workspace),
                                                   _stream_ptr(stream)),
               "compress_lz4")
    return out, nbytes


def compress_noalloc(x: torch.Tensor, elem_size: int, block_size: int = 0,
                     out: torch.Tensor | None = None, nbytes: torch.Tensor | None = None,
                     stream=None):
    """compress (bit transpose + LZ4) through the entry point that allocates
    nothing: the scratch space is the library's fixed per-GPU array, so inputs
    whose workspace_size exceeds NOALLOC_SCRATCH_BYTES are refused.  Calls
    that overlap in time on one GPU race on that array."""
    _require_device(x, out, nbytes)
    total = _nbytes(x)
    if total % elem_size:
        raise ValueError("buffer is not a whole number of elements")
    n = total // elem_size
    if out is None:
        out = torch.empty(compress_bound(n, elem_size, block_size), dtype=torch.uint8,
                          device=x.device)
    if nbytes is None:
        nbytes = torch.empty(1, dtype=torch.int64, device=x.device)
    _check_word(nbytes, torch.int64, "nbytes")
    _lib.check(_lib.lib().bsg_compress_lz4_noalloc(_ptr(x), _ptr(out), n, elem_size, block_size,
                                                    _nbytes(out), _ptr(nbytes),
                                                    _stream_ptr(stream)),
               "compress_lz4_noalloc")
    return out, nbytes


def round_compress(vis: torch.Tensor, autos: torch.Tensor, n_samples: float, f: float,
                   block_size: int = 0, out: torch.Tensor | None = None,
                   workspace: torch.Tensor | None = None, nbytes: torch.Tensor | None = None,
                   prod_map: torch.Tensor | None = None, stream=None):
    """round_to_noise fused into compress (elem_size 4); vis is not modified."""
    _require_device(vis, autos, out, workspace, nbytes, prod_map)
    F, I, T = _vis_autos(vis, autos)
    _check_prod_map(prod_map, vis.shape[1], I)
    n = 2 * vis.numel()
    if out is None:
        out = torch.empty(compress_bound(n, 4, block_size), dtype=torch.uint8, device=vis.device)
    workspace = _alloc_ws(n, 4, block_size, vis.device, workspace)
    if nbytes is None:
        nbytes = torch.empty(1, dtype=torch.int64, device=vis.device)
    _check_word(nbytes, torch.int64, "nbytes")
    _lib.check(_lib.lib().bsg_round_compress_lz4(_ptr(vis), _ptr(autos), F, I, T, _ptr(prod_map),
                                                  float(n_samples), float(f), block_size,
                                                  _ptr(out), _nbytes(out), _ptr(nbytes),
                                                  _ptr(workspace), _nbytes(workspace),
                                                  _stream_ptr(stream)), "round_compress_lz4")
    return out, nbytes


def decompress(stream_bytes: torch.Tensor, in_nbytes: int, n: int, elem_size: int,
               block_size: int = 0, out: torch.Tensor | None = None,
               status: torch.Tensor | None = None, stream=None, filter: int = BSG_FILTER_BIT):
    """Enqueue decompression.  Returns (out, status): status is a device int32
    that reads 0 on success and BSG_ECORRUPT otherwise."""
    _require_device(stream_bytes, out, status)
    if out is None:
        out = torch.empty(max(n * elem_size, 1), dtype=torch.uint8, device=stream_bytes.device)
    _check_out(out, n * elem_size, "decompress")
    if in_nbytes > _nbytes(stream_bytes):
        raise ValueError("in_nbytes exceeds the stream buffer")
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=stream_bytes.device)
    _check_word(status, torch.int32, "status")
    _lib.check(_lib.lib().bsg_decompress_lz4_filter(_ptr(stream_bytes), int(in_nbytes), _ptr(out),
                                                     n, elem_size, block_size, int(filter),
                                                     _ptr(status), _stream_ptr(stream)),
               "decompress_lz4")
    return out, status


def compress_sync(x: torch.Tensor, elem_size: int, block_size: int = 0,
                  filter: int = BSG_FILTER_BIT) -> torch.Tensor:
    out, nb = compress(x, elem_size, block_size, filter=filter)
    m = int(nb.item())
    if m < 0:
        raise BsgError(m, "compress_lz4")
    return out[:m]


def decompress_sync(s: torch.Tensor, n: int, elem_size: int, block_size: int = 0,
                    filter: int = BSG_FILTER_BIT) -> torch.Tensor:
    out, st = decompress(s, _nbytes(s), n, elem_size, block_size, filter=filter)
    code = int(st.item())
    if code != 0:
        raise BsgError(code, "decompress_lz4")
    return out[: n * elem_size]


class BatchPlan:
    """Many chunks, each its own stream, compressed or decompressed by one
    call of the batch C-ABI.  The plan builds the descriptor table (in pinned
    host memory, copied asynchronously to the device on the plan's stream)
    and allocates every buffer once, on that stream; compress() /
    decompress() then only enqueue kernels, so they can be captured into a
    CUDA graph and replayed.  Tensors referenced by the plan are kept alive
    by it.  compress() / decompress() enqueue on the given stream, else the
    current one; work on a stream other than the plan's must be ordered
    after the plan's creation (the table copy)."""

    def __init__(self, rows, device, stream=None):
        L = _lib.lib()
        self.count = len(rows)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._keep = [t for r in rows for t in (r[0], r[2]) if t is not None]
        arr = (_lib.Chunk * max(self.count, 1))()
        for k, (src, in_nbytes, dst, cap, n, e, b) in enumerate(rows):
            arr[k] = _lib.Chunk(src.data_ptr() if src is not None else None, in_nbytes,
                                dst.data_ptr() if dst is not None else None, cap, n, e, b)
        tb = int(L.bsg_batch_table_bytes(self.count))
        self._host_t = torch.empty(tb, dtype=torch.uint8, pin_memory=True)
        self._host = ctypes.c_void_p(self._host_t.data_ptr())
        _lib.check(L.bsg_batch_build_table(arr, self.count, self._host, tb), "batch_build_table")
        with torch.cuda.stream(self.stream):
            self._dev = torch.empty(tb, dtype=torch.uint8, device=device)
            self._dev.copy_(self._host_t, non_blocking=True)
        self.device = device

    @staticmethod
    def _per_chunk(v, k):
        return list(v) if isinstance(v, (list, tuple)) else [v] * k

    @classmethod
    def for_compress(cls, inputs, elem_sizes, block_sizes=0, outs=None, stream=None):
        """inputs: device tensors (any dtype, contiguous) of whole elements;
        outs (optional): uint8 buffers, by default of compress_bound bytes."""
        k = len(inputs)
        es, bs = cls._per_chunk(elem_sizes, k), cls._per_chunk(block_sizes, k)
        _require_device(*inputs)
        device = inputs[0].device if k else torch.device("cuda")
        st = stream if stream is not None else torch.cuda.current_stream(device)
        rows, buf = [], []
        with torch.cuda.stream(st):
            for x, e, b in zip(inputs, es, bs):
                if _nbytes(x) % e:
                    raise ValueError("buffer is not a whole number of elements")
                n = _nbytes(x) // e
                buf.append(torch.empty(compress_bound(n, e, b), dtype=torch.uint8, device=device)
                           if outs is None else outs[len(buf)])
                rows.append((x, 0, buf[-1], _nbytes(buf[-1]), n, e, b))
            plan = cls(rows, device, st)
            plan.outs = buf
            plan.meta = [(r[4], r[5], r[6]) for r in rows]
            ws = int(_lib.lib().bsg_batch_workspace_size(plan._host))
            plan.workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=device)
            plan.nbytes = torch.zeros(max(k, 1), dtype=torch.int64, device=device)
        return plan

    @classmethod
    def for_decompress(cls, streams, in_nbytes, ns, elem_sizes, block_sizes=0, outs=None,
                       stream=None):
        """streams: device uint8 tensors holding the streams; in_nbytes their
        lengths; ns the element counts; outs (optional) the destinations."""
        k = len(streams)
        es, bs = cls._per_chunk(elem_sizes, k), cls._per_chunk(block_sizes, k)
        _require_device(*streams)
        device = streams[0].device if k else torch.device("cuda")
        st = stream if stream is not None else torch.cuda.current_stream(device)
        rows, buf = [], []
        with torch.cuda.stream(st):
            for s, m, n, e, b in zip(streams, in_nbytes, ns, es, bs):
                buf.append(torch.empty(max(n * e, 1), dtype=torch.uint8, device=device)
                           if outs is None else outs[len(buf)])
                rows.append((s, int(m), buf[-1], 0, int(n), e, b))
            plan = cls(rows, device, st)
            plan.outs = buf
            plan.meta = [(r[4], r[5], r[6]) for r in rows]
            plan.status = torch.zeros(max(k, 1), dtype=torch.int32, device=device)
        return plan

    def compress(self, waves_per_cu: int = 0, schedule: int = BSG_SCHED_STRIDED,
                 stream=None) -> torch.Tensor:
        """Enqueue; returns the device int64 stream lengths (caller's order).
        waves_per_cu and schedule set the launch shape (never the bytes)."""
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        _lib.check(_lib.lib().bsg_batch_compress(self._host, _ptr(self._dev), _ptr(self.nbytes),
                                                  _ptr(self.workspace), _nbytes(self.workspace),
                                                  int(waves_per_cu), int(schedule),
                                                  _stream_ptr(st)),
                   "batch_compress")
        return self.nbytes

    def decompress(self, waves_per_cu: int = 0, schedule: int = BSG_SCHED_STRIDED,
                   stream=None) -> torch.Tensor:
        """Enqueue; returns the device int32 per-chunk status (0 = ok)."""
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.stream(st):
            self.status.zero_()
        _lib.check(_lib.lib().bsg_batch_decompress(self._host, _ptr(self._dev), _ptr(self.status),
                                                    int(waves_per_cu), int(schedule),
                                                    _stream_ptr(st)),
                   "batch_decompress")
        return self.status


def read_header(host_bytes: bytes) -> Header:
    h = Header()
    buf = ctypes.create_string_buffer(bytes(host_bytes[:24]), 24)
    _lib.check(_lib.lib().bsg_read_header(buf, len(host_bytes), ctypes.byref(h)), "read_header")
    return h
