"""The system liblz4 (1.9.x), called through its public C API as a black box.

Test-only: an LZ4 block decoder and encoder that is independent of both the
oracle and the GPU library.  Never a product dependency."""
import ctypes
import ctypes.util

import numpy as np

_lib = None


def available() -> bool:
    try:
        lib()
        return True
    except OSError:
        return False


def lib():
    global _lib
    if _lib is None:
        name = ctypes.util.find_library("lz4") or "liblz4.so.1"
        L = ctypes.CDLL(name)
        L.LZ4_decompress_safe.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int, ctypes.c_int]
        L.LZ4_decompress_safe.restype = ctypes.c_int
        L.LZ4_compress_default.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int, ctypes.c_int]
        L.LZ4_compress_default.restype = ctypes.c_int
        L.LZ4_compress_HC.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.LZ4_compress_HC.restype = ctypes.c_int
        L.LZ4_compressBound.argtypes = [ctypes.c_int]
        L.LZ4_compressBound.restype = ctypes.c_int
        _lib = L
    return _lib


def decompress_safe(comp: bytes, n_out: int):
    """Decoded bytes, or None when liblz4 reports an error or a size mismatch."""
    dst = ctypes.create_string_buffer(max(n_out, 1))
    r = lib().LZ4_decompress_safe(bytes(comp), dst, len(comp), n_out)
    if r != n_out:
        return None
    return dst.raw[:n_out]


def compress_default(data: bytes) -> bytes:
    cap = lib().LZ4_compressBound(len(data))
    dst = ctypes.create_string_buffer(cap)
    r = lib().LZ4_compress_default(bytes(data), dst, len(data), cap)
    assert r > 0
    return dst.raw[:r]


def compress_hc(data: bytes, level: int = 9) -> bytes:
    cap = lib().LZ4_compressBound(len(data))
    dst = ctypes.create_string_buffer(cap)
    r = lib().LZ4_compress_HC(bytes(data), dst, len(data), cap, level)
    assert r > 0
    return dst.raw[:r]


def parse_sequences(comp: bytes):
    """Split an LZ4 block into (literals, offset, match_len) triples; the last
    triple has offset None.  Raises ValueError on malformed input."""
    b = memoryview(bytes(comp))
    ip = 0
    out = []
    while True:
        if ip >= len(b):
            raise ValueError("missing token")
        tok = b[ip]
        ip += 1
        ll = tok >> 4
        if ll == 15:
            while True:
                x = b[ip]
                ip += 1
                ll += x
                if x != 255:
                    break
        lit = bytes(b[ip:ip + ll])
        if len(lit) != ll:
            raise ValueError("literals run past the end")
        ip += ll
        if ip == len(b):
            out.append((lit, None, 0))
            return out
        off = b[ip] | (b[ip + 1] << 8)
        ip += 2
        ml = (tok & 15) + 4
        if (tok & 15) == 15:
            while True:
                x = b[ip]
                ip += 1
                ml += x
                if x != 255:
                    break
        out.append((lit, off, ml))
