"""CPU oracle for the compression scheme of arXiv:1503.00638.

TEST INFRASTRUCTURE ONLY: the plain C statement of what the GPU path must
compute (oracle.c), loaded through ctypes.  Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import this package; the
product library never does.  It imports nothing from the product package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# -O2 without fast-math and without FMA contraction: the rounding step is
# defined in plain IEEE double arithmetic.
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (next to the source)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        i64, i32, dbl, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        L.oracle_round_to_noise.argtypes = [vp, vp, vp, i64, i64, i64, vp, dbl, dbl, i32]
        L.oracle_round_to_noise.restype = i32
        L.oracle_granularity_exponent.argtypes = [dbl]
        L.oracle_granularity_exponent.restype = i32
        L.oracle_round_to_multiple.argtypes = [ctypes.c_float, i32]
        L.oracle_round_to_multiple.restype = ctypes.c_float
        L.oracle_round_int_to_multiple.argtypes = [ctypes.c_int32, i32]
        L.oracle_round_int_to_multiple.restype = ctypes.c_int32
        L.oracle_round_to_noise_i32.argtypes = [vp, vp, vp, i64, i64, i64, vp, dbl, dbl, i32]
        L.oracle_round_to_noise_i32.restype = i32
        L.oracle_noise_compensation.argtypes = [vp, vp, i64, i64, i64, vp, vp]
        L.oracle_noise_compensation.restype = i32
        L.oracle_round_to_noise_scaled.argtypes = [vp, vp, vp, i64, i64, i64, vp, dbl, dbl, vp, i32]
        L.oracle_round_to_noise_scaled.restype = i32
        for name in ("oracle_bitshuffle", "oracle_bitunshuffle"):
            getattr(L, name).argtypes = [vp, vp, i64, i64, i64, i32]
            getattr(L, name).restype = i32
        L.oracle_lz4_compress_block.argtypes = [vp, i64, vp, i64]
        L.oracle_lz4_compress_block.restype = i64
        L.oracle_lz4_decompress_block.argtypes = [vp, i64, vp, i64]
        L.oracle_lz4_decompress_block.restype = i64
        L.oracle_block_elems.argtypes = [i64, i64]
        L.oracle_block_elems.restype = i64
        L.oracle_compress_bound.argtypes = [i64, i64, i64]
        L.oracle_compress_bound.restype = i64
        L.oracle_compress.argtypes = [vp, vp, i64, i64, i64, i64, i32]
        L.oracle_compress.restype = i64
        L.oracle_decompress.argtypes = [vp, i64, vp, i64, i64, i64, i32]
        L.oracle_decompress.restype = i64
        for name in ("oracle_byteshuffle", "oracle_byteunshuffle"):
            getattr(L, name).argtypes = [vp, vp, i64, i64, i64, i32]
            getattr(L, name).restype = i32
        L.oracle_compress_filter.argtypes = [vp, vp, i64, i64, i64, i32, i64, i32]
        L.oracle_compress_filter.restype = i64
        L.oracle_decompress_filter.argtypes = [vp, i64, vp, i64, i64, i64, i32, i32]
        L.oracle_decompress_filter.restype = i64
        L.oracle_fullcov_inverse_diag.argtypes = [vp, vp, i64, i64, i64, vp]
        L.oracle_fullcov_inverse_diag.restype = i32
        L.oracle_round_to_noise_fullcov.argtypes = [vp, vp, vp, i64, i64, i64, dbl, dbl]
        L.oracle_round_to_noise_fullcov.restype = i32
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = i32
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


def _as_u8(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a)
    return a.view(np.uint8).reshape(-1)


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def granularity_exponent(G2: float) -> int:
    return int(lib().oracle_granularity_exponent(float(G2)))


def round_to_multiple(x: float, k: int) -> float:
    return float(np.float32(lib().oracle_round_to_multiple(float(x), int(k))))


def round_to_noise(vis: np.ndarray, autos: np.ndarray, n_samples: float, f: float,
                   prod_map: np.ndarray | None = None, nthreads: int = 0) -> np.ndarray:
    """vis complex64 (F, P, T), autos float32 (F, I, T) -> rounded copy of vis."""
    vis = np.ascontiguousarray(vis, dtype=np.complex64)
    autos = np.ascontiguousarray(autos, dtype=np.float32)
    F, I, T = autos.shape
    if vis.shape != (F, I * (I + 1) // 2, T):
        raise ValueError(f"vis shape {vis.shape} does not match autos {autos.shape}")
    out = np.empty_like(vis)
    pm = None if prod_map is None else np.ascontiguousarray(prod_map, dtype=np.int32)
    rc = lib().oracle_round_to_noise(_ptr(vis), _ptr(out), _ptr(autos), F, I, T, _ptr(pm),
                                     float(n_samples), float(f), int(nthreads))
    if rc != 0:
        raise OracleError(rc, "round_to_noise")
    return out


def noise_compensation(vis: np.ndarray, autos: np.ndarray,
                       prod_map: np.ndarray | None = None) -> np.ndarray:
    """Per-(frequency, time) compensation factor (F, T) float64."""
    vis = np.ascontiguousarray(vis, dtype=np.complex64)
    autos = np.ascontiguousarray(autos, dtype=np.float32)
    F, I, T = autos.shape
    if vis.shape != (F, I * (I + 1) // 2, T):
        raise ValueError(f"vis shape {vis.shape} does not match autos {autos.shape}")
    out = np.empty((F, T), dtype=np.float64)
    pm = None if prod_map is None else np.ascontiguousarray(prod_map, dtype=np.int32)
    rc = lib().oracle_noise_compensation(_ptr(vis), _ptr(autos), F, I, T, _ptr(pm), _ptr(out))
    if rc != 0:
        raise OracleError(rc, "noise_compensation")
    return out


def round_to_noise_scaled(vis: np.ndarray, autos: np.ndarray, n_samples: float, f: float,
                          scale: np.ndarray, prod_map: np.ndarray | None = None,
                          nthreads: int = 0) -> np.ndarray:
    vis = np.ascontiguousarray(vis, dtype=np.complex64)
    autos = np.ascontiguousarray(autos, dtype=np.float32)
    F, I, T = autos.shape
    scale = np.ascontiguousarray(scale, dtype=np.float64)
    if vis.shape != (F, I * (I + 1) // 2, T) or scale.shape != (F, T):
        raise ValueError("shape mismatch")
    out = np.empty_like(vis)
    pm = None if prod_map is None else np.ascontiguousarray(prod_map, dtype=np.int32)
    rc = lib().oracle_round_to_noise_scaled(_ptr(vis), _ptr(out), _ptr(autos), F, I, T, _ptr(pm),
                                            float(n_samples), float(f), _ptr(scale), int(nthreads))
    if rc != 0:
        raise OracleError(rc, "round_to_noise_scaled")
    return out


def fullcov_inverse_diag(vis: np.ndarray, autos: np.ndarray) -> np.ndarray:
    """(F, T, I^2) float64: (Q^-1)_kk per degree of freedom, Q = 2N C."""
    vis = np.ascontiguousarray(vis, dtype=np.complex64)
    autos = np.ascontiguousarray(autos, dtype=np.float32)
    F, I, T = autos.shape
    if vis.shape != (F, I * (I + 1) // 2, T):
        raise ValueError("shape mismatch")
    out = np.empty((F, T, I * I), dtype=np.float64)
    rc = lib().oracle_fullcov_inverse_diag(_ptr(vis), _ptr(autos), F, I, T, _ptr(out))
    if rc != 0:
        raise OracleError(rc, "fullcov_inverse_diag")
    return out


def round_to_noise_fullcov(vis: np.ndarray, autos: np.ndarray, n_samples: float,
                           f: float) -> np.ndarray:
    vis = np.ascontiguousarray(vis, dtype=np.complex64)
    autos = np.ascontiguousarray(autos, dtype=np.float32)
    F, I, T = autos.shape
    out = np.empty_like(vis)
    rc = lib().oracle_round_to_noise_fullcov(_ptr(vis), _ptr(out), _ptr(autos), F, I, T,
                                             float(n_samples), float(f))
    if rc != 0:
        raise OracleError(rc, "round_to_noise_fullcov")
    return out


def round_int_to_multiple(x: int, k: int) -> int:
    return int(lib().oracle_round_int_to_multiple(int(x), int(k)))


def round_to_noise_i32(vis: np.ndarray, autos: np.ndarray, n_samples: float, f: float,
                       prod_map: np.ndarray | None = None, nthreads: int = 0) -> np.ndarray:
    """vis int32 (F, P, T, 2), autos int32 (F, I, T) -> rounded copy of vis."""
    vis = np.ascontiguousarray(vis, dtype=np.int32)
    autos = np.ascontiguousarray(autos, dtype=np.int32)
    F, I, T = autos.shape
    if vis.shape != (F, I * (I + 1) // 2, T, 2):
        raise ValueError(f"vis shape {vis.shape} does not match autos {autos.shape}")
    out = np.empty_like(vis)
    pm = None if prod_map is None else np.ascontiguousarray(prod_map, dtype=np.int32)
    rc = lib().oracle_round_to_noise_i32(_ptr(vis), _ptr(out), _ptr(autos), F, I, T, _ptr(pm),
                                         float(n_samples), float(f), int(nthreads))
    if rc != 0:
        raise OracleError(rc, "round_to_noise_i32")
    return out


def block_elems(elem_size: int, block_size: int = 0) -> int:
    return int(lib().oracle_block_elems(elem_size, block_size))


def _transpose(fn, data, elem_size, block_size, nthreads):
    src = _as_u8(data)
    if src.size % elem_size:
        raise ValueError("buffer is not a whole number of elements")
    out = np.empty_like(src)
    rc = fn(_ptr(src), _ptr(out), src.size // elem_size, elem_size, block_size, nthreads)
    if rc != 0:
        raise OracleError(rc, fn.__name__)
    return out


def bitshuffle(data: np.ndarray, elem_size: int, block_size: int = 0, nthreads: int = 0) -> np.ndarray:
    return _transpose(lib().oracle_bitshuffle, data, elem_size, block_size, nthreads)


def bitunshuffle(data: np.ndarray, elem_size: int, block_size: int = 0, nthreads: int = 0) -> np.ndarray:
    return _transpose(lib().oracle_bitunshuffle, data, elem_size, block_size, nthreads)


def byteshuffle(data: np.ndarray, elem_size: int, block_size: int = 0, nthreads: int = 0) -> np.ndarray:
    return _transpose(lib().oracle_byteshuffle, data, elem_size, block_size, nthreads)


def byteunshuffle(data: np.ndarray, elem_size: int, block_size: int = 0, nthreads: int = 0) -> np.ndarray:
    return _transpose(lib().oracle_byteunshuffle, data, elem_size, block_size, nthreads)


def lz4_compress_block(block: np.ndarray) -> bytes:
    src = _as_u8(block)
    cap = src.size + src.size // 255 + 16
    dst = np.empty(cap, dtype=np.uint8)
    n = lib().oracle_lz4_compress_block(_ptr(src), src.size, _ptr(dst), cap)
    if n < 0:
        raise OracleError(n, "lz4_compress_block")
    return dst[:n].tobytes()


def lz4_decompress_block(comp: bytes, n_out: int) -> bytes:
    src = np.frombuffer(bytes(comp), dtype=np.uint8)
    dst = np.empty(max(n_out, 1), dtype=np.uint8)
    n = lib().oracle_lz4_decompress_block(_ptr(src), src.size, _ptr(dst), n_out)
    if n < 0:
        raise OracleError(n, "lz4_decompress_block")
    return dst[:n_out].tobytes()


def compress_bound(n: int, elem_size: int, block_size: int = 0) -> int:
    return int(lib().oracle_compress_bound(n, elem_size, block_size))


def compress(data: np.ndarray, elem_size: int, block_size: int = 0, nthreads: int = 0,
             filter: int = 0) -> np.ndarray:
    """Stream of data; filter 0 = bit transpose (the method), 1 = byte shuffle."""
    src = _as_u8(data)
    n = src.size // elem_size
    if n * elem_size != src.size:
        raise ValueError("buffer is not a whole number of elements")
    cap = compress_bound(n, elem_size, block_size)
    if cap < 0:
        raise OracleError(cap, "compress_bound")
    out = np.empty(cap, dtype=np.uint8)
    m = lib().oracle_compress_filter(_ptr(src), _ptr(out), n, elem_size, block_size, int(filter),
                                     cap, nthreads)
    if m < 0:
        raise OracleError(m, "compress")
    return out[:m]


def decompress(stream: np.ndarray, n: int, elem_size: int, block_size: int = 0,
               nthreads: int = 0, filter: int = 0) -> np.ndarray:
    src = _as_u8(stream)
    out = np.empty(max(n * elem_size, 1), dtype=np.uint8)
    rc = lib().oracle_decompress_filter(_ptr(src), src.size, _ptr(out), n, elem_size, block_size,
                                        int(filter), nthreads)
    if rc != 0:
        raise OracleError(rc, "decompress")
    return out[: n * elem_size]
