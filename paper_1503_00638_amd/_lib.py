"""ctypes binding of libbsg.so (the C-ABI declared in include/bsg.h).

Argument marshalling only: every step runs in the HIP library.  Loading
fails loudly when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbsg.so")

BSG_OK = 0
BSG_FILTER_BIT, BSG_FILTER_BYTE = 0, 1
BSG_SCHED_STRIDED, BSG_SCHED_RANGES = 0, 1
BSG_EINVAL = -1
BSG_ECAPACITY = -2
BSG_ECORRUPT = -3
BSG_EHIP = -4
MAGIC = 0x31475342

EXPORTS = (
    "bsg_strerror", "bsg_block_elems", "bsg_round_to_noise", "bsg_bitshuffle",
    "bsg_bitunshuffle", "bsg_compress_bound", "bsg_compress_workspace_size",
    "bsg_compress_lz4", "bsg_round_compress_lz4", "bsg_decompress_lz4", "bsg_read_header",
    "bsg_batch_table_bytes", "bsg_batch_build_table", "bsg_batch_workspace_size",
    "bsg_batch_compress", "bsg_batch_decompress", "bsg_round_to_noise_i32",
    "bsg_noise_compensation", "bsg_round_to_noise_scaled", "bsg_byteshuffle",
    "bsg_byteunshuffle", "bsg_compress_lz4_filter", "bsg_decompress_lz4_filter",
    "bsg_fullcov_inverse_diag", "bsg_round_to_noise_fullcov", "bsg_compress_lz4_noalloc",
)
NOALLOC_SCRATCH_BYTES = 64 << 20


class Header(ctypes.Structure):
    _fields_ = [("magic", ctypes.c_uint32), ("elem_size", ctypes.c_uint32),
                ("n", ctypes.c_uint64), ("block_elems", ctypes.c_uint32),
                ("n_blocks", ctypes.c_uint32)]


class Chunk(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p), ("in_nbytes", ctypes.c_int64),
                ("out", ctypes.c_void_p), ("out_capacity", ctypes.c_int64),
                ("n", ctypes.c_int64), ("elem_size", ctypes.c_int64),
                ("block_size", ctypes.c_int64)]


class BsgError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = _lib().bsg_strerror(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1503_00638_amd.build` "
                "(or __graft_entry__.build()); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.bsg_strerror.argtypes = [i32]
        L.bsg_strerror.restype = ctypes.c_char_p
        L.bsg_block_elems.argtypes = [i64, i64]
        L.bsg_block_elems.restype = i64
        L.bsg_round_to_noise.argtypes = [vp, vp, vp, i64, i64, i64, vp, dbl, dbl, vp]
        L.bsg_round_to_noise.restype = i32
        L.bsg_round_to_noise_i32.argtypes = [vp, vp, vp, i64, i64, i64, vp, dbl, dbl, vp]
        L.bsg_round_to_noise_i32.restype = i32
        L.bsg_noise_compensation.argtypes = [vp, vp, i64, i64, i64, vp, vp, vp]
        L.bsg_noise_compensation.restype = i32
        L.bsg_round_to_noise_scaled.argtypes = [vp, vp, vp, i64, i64, i64, vp, dbl, dbl, vp, vp]
        L.bsg_round_to_noise_scaled.restype = i32
        L.bsg_fullcov_inverse_diag.argtypes = [vp, vp, i64, i64, i64, vp, vp]
        L.bsg_fullcov_inverse_diag.restype = i32
        L.bsg_round_to_noise_fullcov.argtypes = [vp, vp, vp, i64, i64, i64, dbl, dbl, vp]
        L.bsg_round_to_noise_fullcov.restype = i32
        for f in (L.bsg_bitshuffle, L.bsg_bitunshuffle, L.bsg_byteshuffle, L.bsg_byteunshuffle):
            f.argtypes = [vp, vp, i64, i64, i64, vp]
            f.restype = i32
        L.bsg_compress_bound.argtypes = [i64, i64, i64]
        L.bsg_compress_bound.restype = i64
        L.bsg_compress_workspace_size.argtypes = [i64, i64, i64]
        L.bsg_compress_workspace_size.restype = i64
        L.bsg_compress_lz4.argtypes = [vp, vp, i64, i64, i64, i64, vp, vp, i64, vp]
        L.bsg_compress_lz4.restype = i32
        L.bsg_compress_lz4_noalloc.argtypes = [vp, vp, i64, i64, i64, i64, vp, vp]
        L.bsg_compress_lz4_noalloc.restype = i32
        L.bsg_round_compress_lz4.argtypes = [vp, vp, i64, i64, i64, vp, dbl, dbl, i64, vp, i64,
                                             vp, vp, i64, vp]
        L.bsg_round_compress_lz4.restype = i32
        L.bsg_decompress_lz4.argtypes = [vp, i64, vp, i64, i64, i64, vp, vp]
        L.bsg_decompress_lz4.restype = i32
        L.bsg_compress_lz4_filter.argtypes = [vp, vp, i64, i64, i64, ctypes.c_int32, i64, vp, vp, i64,
                                              vp]
        L.bsg_compress_lz4_filter.restype = i32
        L.bsg_decompress_lz4_filter.argtypes = [vp, i64, vp, i64, i64, i64, ctypes.c_int32, vp, vp]
        L.bsg_decompress_lz4_filter.restype = i32
        L.bsg_read_header.argtypes = [vp, i64, ctypes.POINTER(Header)]
        L.bsg_read_header.restype = i32
        L.bsg_batch_table_bytes.argtypes = [ctypes.c_int32]
        L.bsg_batch_table_bytes.restype = i64
        L.bsg_batch_build_table.argtypes = [ctypes.POINTER(Chunk), ctypes.c_int32, vp, i64]
        L.bsg_batch_build_table.restype = i32
        L.bsg_batch_workspace_size.argtypes = [vp]
        L.bsg_batch_workspace_size.restype = i64
        L.bsg_batch_compress.argtypes = [vp, vp, vp, vp, i64, ctypes.c_int32, ctypes.c_int32, vp]
        L.bsg_batch_compress.restype = i32
        L.bsg_batch_decompress.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_int32, vp]
        L.bsg_batch_decompress.restype = i32
        _LIB = L
    return _LIB


def lib():
    return _lib()


def check(code: int, what: str) -> None:
    if code != BSG_OK:
        raise BsgError(code, what)
