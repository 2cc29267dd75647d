"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no noise estimate, no rounding, no transpose, no LZ4).
Both the HIP path and the CPU oracle consume what it returns, so it is the one
piece of code the two sides share.

Stand-in for the CHIME Pathfinder data of Section 5 (not available here):

* visibilities are a (freq, product, time) array, time fastest (Section 2
  "time minor" and Section 5 layout); products are all pairs i <= j of the
  inputs, autos included, ordered upper-triangle row-major;
* auto-correlations are positive smooth spectra around 1e3 (+-20% over
  frequency, +-2% over time), each with its radiometer scatter
  V_ii / sqrt(N) added to the real part, imaginary part exactly zero;
* cross-correlations are noise dominated: real and imaginary parts are
  independent normals of variance V_ii V_jj / (2N), the diagonal radiometer
  variance of Section 3.1;
* N = 3.9e6 samples per integration (0.39 MHz x 10 s, the binning of the
  paper's example figure).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

N_SAMPLES_DEFAULT = 3.9e6


def n_products(n_inputs: int) -> int:
    return n_inputs * (n_inputs + 1) // 2


def product_pairs(n_inputs: int) -> np.ndarray:
    """(P, 2) int32 table of (i, j), i <= j, upper-triangle row-major."""
    out = np.empty((n_products(n_inputs), 2), dtype=np.int32)
    p = 0
    for i in range(n_inputs):
        m = n_inputs - i
        out[p:p + m, 0] = i
        out[p:p + m, 1] = np.arange(i, n_inputs, dtype=np.int32)
        p += m
    return out


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def auto_model(F: int, I: int, T: int, rng: np.random.Generator) -> np.ndarray:
    """Noise-free auto-correlation power, float64 (F, I, T)."""
    phi = rng.random(I)
    psi = rng.random(I)
    f = np.arange(F)[:, None, None]
    t = np.arange(T)[None, None, :]
    spec = 1.0 + 0.2 * np.sin(2 * np.pi * (f / F + phi[None, :, None]))
    tvar = 1.0 + 0.02 * np.sin(2 * np.pi * (t / T + psi[None, :, None]))
    return 1e3 * spec * tvar


def gen_vis(F: int, I: int, T: int, seed: int, n_samples: float = N_SAMPLES_DEFAULT):
    """Return (vis, autos): vis complex64 (F, P, T), autos float32 (F, I, T).

    autos are the real parts of the auto products as stored (the measured
    autos, pre-rounding), which is what the noise estimate is computed from.
    Generated one frequency at a time from one PCG64 stream so that large
    shapes never hold more than one frequency of float64 scratch.
    """
    rng = _rng(seed)
    A = auto_model(F, I, T, rng)  # float64 (F, I, T); 16 MiB at the largest config
    P = n_products(I)
    pairs = product_pairs(I)
    ii, jj = pairs[:, 0], pairs[:, 1]
    is_auto = ii == jj
    vis = np.empty((F, P, T), dtype=np.complex64)
    vf = vis.view(np.float32).reshape(F, P, T, 2)
    inv_sqrt_n = 1.0 / math.sqrt(n_samples)
    for f in range(F):
        Af = A[f]  # (I, T)
        z = rng.standard_normal((P, T, 2), dtype=np.float32)
        # cross: sigma = sqrt(A_i A_j / (2N)) for re and im separately
        sig = np.sqrt(Af[ii] * Af[jj] * (0.5 / n_samples)).astype(np.float32)
        vf[f, :, :, 0] = z[:, :, 0] * sig
        vf[f, :, :, 1] = z[:, :, 1] * sig
        # autos: A + N(0, A^2/N) on the real part, imaginary exactly zero
        Aa = Af[ii[is_auto]]
        vf[f, is_auto, :, 0] = (Aa + Aa * inv_sqrt_n * z[is_auto, :, 0]).astype(np.float32)
        vf[f, is_auto, :, 1] = 0.0
    autos = np.ascontiguousarray(vf[..., 0][:, is_auto, :])  # (F, I, T) float32
    return vis, autos


def gen_vis_point_source(F: int, I: int, T: int, seed: int, source: float = 0.4,
                         n_samples: float = N_SAMPLES_DEFAULT):
    """Visibilities dominated by one unresolved source at zenith with
    calibrated gains (the case Section 3.1 uses to show correlated noise):
    every product gains the same real term S = source x the mean receiver
    power, autos included, on top of the noise model above.  Returns
    (vis complex64 (F, P, T), autos float32 (F, I, T))."""
    vis, _ = gen_vis(F, I, T, seed, n_samples)
    vf = vis.view(np.float32).reshape(F, -1, T, 2)
    vf[..., 0] += np.float32(source * 1e3)
    pairs = product_pairs(I)
    is_auto = pairs[:, 0] == pairs[:, 1]
    autos = np.ascontiguousarray(vf[..., 0][:, is_auto, :])
    return vis, autos


def gen_vis_int(F: int, I: int, T: int, seed: int, n_samples: float = N_SAMPLES_DEFAULT,
                scale: float = 1024.0):
    """Integer visibilities, the data type of the paper's correlator output:
    the model above scaled by `scale` and rounded to integers.  Returns
    (vis int32 (F, P, T, 2), autos int32 (F, I, T)), autos being the real
    parts of the auto products."""
    vis, _ = gen_vis(F, I, T, seed, n_samples)
    vi = np.rint(vis.view(np.float32).reshape(F, -1, T, 2).astype(np.float64) * scale)
    vi = vi.astype(np.int32)
    pairs = product_pairs(I)
    is_auto = pairs[:, 0] == pairs[:, 1]
    autos = np.ascontiguousarray(vi[..., 0][:, is_auto, :])
    return vi, autos


# ---------------------------------------------------------------------------
# bit-transpose sweep inputs
# ---------------------------------------------------------------------------

def gen_uniform_bytes(nbytes: int, seed: int) -> np.ndarray:
    return _rng(seed).integers(0, 256, size=nbytes, dtype=np.uint8)


def gen_gauss_int32(n: int, k: int, seed: int) -> np.ndarray:
    """int32 values round(N(0, sigma=2**k)): low-bit entropy set by k."""
    z = _rng(seed).standard_normal(n)
    return np.rint(z * float(2 ** k)).astype(np.int32)


# ---------------------------------------------------------------------------
# batched chunks
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class ChunkSpec:
    index: int
    nbytes: int
    elem_size: int
    kind: str  # "vis" or "walk"
    seed: int

    @property
    def n(self) -> int:
        return self.nbytes // self.elem_size


def gen_batch_specs(count: int = 4096, seed: int = 3, lo: int = 1 << 16, hi: int = 1 << 26,
                    elem_sizes=(2, 4, 8)) -> list[ChunkSpec]:
    """Chunk sizes log-uniform in [lo, hi) bytes, rounded down to a multiple of
    the element size; element size and content kind drawn per chunk."""
    rng = _rng(seed)
    out = []
    for c in range(count):
        nb = int(math.exp(rng.uniform(math.log(lo), math.log(hi))))
        e = int(rng.choice(np.asarray(elem_sizes)))
        nb -= nb % e
        kind = "vis" if rng.random() < 0.5 else "walk"
        out.append(ChunkSpec(c, nb, e, kind, seed + 1 + c))
    return out


def gen_walk_int16(n: int, seed: int) -> np.ndarray:
    """int16 random walk from 0, steps uniform in [-8, 8], int16 wraparound."""
    steps = _rng(seed).integers(-8, 9, size=n, dtype=np.int64)
    return (np.cumsum(steps) & 0xFFFF).astype(np.uint16).view(np.int16)


def gen_short_matches(nbytes: int, seed: int, lit_max: int = 4, match_lo: int = 12,
                      match_hi: int = 18, window: int = 600) -> np.ndarray:
    """Bytes built as an LZ77 source: runs of 0..lit_max random literals, each
    followed by a copy of match_lo..match_hi bytes from up to `window` bytes
    back.  An 8 KiB block of it parses into hundreds of short sequences."""
    rng = _rng(seed)
    out = bytearray(rng.integers(0, 256, 16, dtype=np.uint8).tobytes())
    while len(out) < nbytes:
        out += rng.integers(0, 256, int(rng.integers(0, lit_max + 1)), dtype=np.uint8).tobytes()
        ln = int(rng.integers(match_lo, match_hi + 1))
        src = len(out) - int(rng.integers(1, min(window, len(out)) + 1))
        for k in range(ln):  # byte by byte: overlapping copies repeat a period
            out.append(out[src + k])
    return np.frombuffer(bytes(out[:nbytes]), dtype=np.uint8).copy()


def gen_chunk_bytes(spec: ChunkSpec, vis_inputs: int = 16) -> np.ndarray:
    """Raw (pre-rounding) chunk content as uint8 of exactly spec.nbytes.

    "vis" chunks are complex64 visibilities from gen_vis at `vis_inputs`
    inputs with as many frequencies as needed; the caller rounds them (each
    side with its own round_to_noise) via gen_chunk_vis when it wants the
    rounded content.
    """
    if spec.kind == "walk":
        w = gen_walk_int16((spec.nbytes + 1) // 2, spec.seed)
        return w.view(np.uint8)[: spec.nbytes].copy()
    vis, _ = gen_chunk_vis(spec, vis_inputs)
    return vis.view(np.uint8).reshape(-1)[: spec.nbytes].copy()


def gen_chunk_vis(spec: ChunkSpec, vis_inputs: int = 16, T: int = 32):
    """(vis, autos) covering at least spec.nbytes bytes of complex64."""
    P = n_products(vis_inputs)
    per_f = P * T * 8
    F = max(1, -(-spec.nbytes // per_f))
    return gen_vis(F, vis_inputs, T, spec.seed)


# ---------------------------------------------------------------------------
# device-side generators (torch RNG on the GPU) for the large workloads
# ---------------------------------------------------------------------------
# The same models as above, drawn with torch's device generator so that tens
# of GiB are produced in seconds.  Bit patterns differ from the numpy
# generators (a different RNG), the distributions are the same.  A check
# against the oracle copies the generated raw input to the host.

def gen_vis_device(F: int, I: int, T: int, seed: int, n_samples: float = N_SAMPLES_DEFAULT,
                   device="cuda"):
    """(vis complex64 (F, P, T), autos float32 (F, I, T)) on the device."""
    import torch
    g = torch.Generator(device=device).manual_seed(int(seed))
    f64 = torch.float64
    phi = torch.rand(I, generator=g, device=device, dtype=f64)
    psi = torch.rand(I, generator=g, device=device, dtype=f64)
    f = torch.arange(F, device=device, dtype=f64)[:, None, None]
    t = torch.arange(T, device=device, dtype=f64)[None, None, :]
    A = 1e3 * (1.0 + 0.2 * torch.sin(2 * math.pi * (f / F + phi[None, :, None]))) * \
        (1.0 + 0.02 * torch.sin(2 * math.pi * (t / T + psi[None, :, None])))
    pairs = torch.from_numpy(product_pairs(I)).to(device=device, dtype=torch.long)
    ii, jj = pairs[:, 0], pairs[:, 1]
    is_auto = ii == jj
    z = torch.randn((F, pairs.shape[0], T, 2), generator=g, device=device, dtype=torch.float32)
    sig = torch.sqrt(A[:, ii] * A[:, jj] * (0.5 / n_samples)).to(torch.float32)
    vf = z * sig[..., None]
    del sig
    Aa = A[:, ii[is_auto]]
    vf[:, is_auto, :, 0] = (Aa + Aa * (1.0 / math.sqrt(n_samples)) * z[:, is_auto, :, 0]).to(torch.float32)
    vf[:, is_auto, :, 1] = 0.0
    del z
    autos = vf[:, is_auto, :, 0].contiguous()
    return torch.view_as_complex(vf), autos


def gen_walk_device(n: int, seed: int, device="cuda"):
    """int16 random walk from 0 (steps uniform in [-8, 8], wraparound)."""
    import torch
    g = torch.Generator(device=device).manual_seed(int(seed))
    steps = torch.randint(-8, 9, (n,), generator=g, device=device, dtype=torch.int32)
    w = torch.cumsum(steps, 0, dtype=torch.int32)
    return (((w + 32768) & 0xFFFF) - 32768).to(torch.int16)


def gen_chunk_vis_device(spec: ChunkSpec, vis_inputs: int = 16, T: int = 32, device="cuda"):
    """Device (vis, autos) covering at least spec.nbytes bytes of complex64."""
    per_f = n_products(vis_inputs) * T * 8
    F = max(1, -(-spec.nbytes // per_f))
    return gen_vis_device(F, vis_inputs, T, spec.seed, device=device)


def gen_walk_chunk_device(spec: ChunkSpec, device="cuda"):
    """Device uint8 tensor of spec.nbytes bytes of int16 random walk."""
    import torch
    w = gen_walk_device((spec.nbytes + 1) // 2, spec.seed, device)
    return w.view(torch.uint8)[: spec.nbytes]


# ---------------------------------------------------------------------------
# serving requests
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Request:
    rid: int
    t_arrival: float  # seconds from start
    op: str  # "compress" | "decompress"
    payload: int  # index into the payload pool
    nbytes: int  # uncompressed bytes (the payload's size)


def gen_pool_sizes(count: int = 256, seed: int = 4, lo: int = 1 << 18, hi: int = 1 << 28,
                   elem_size: int = 4) -> list[int]:
    """Payload sizes log-uniform in [lo, hi) bytes, whole elements."""
    rng = _rng(seed)
    out = []
    for _ in range(count):
        nb = int(math.exp(rng.uniform(math.log(lo), math.log(hi))))
        out.append(nb - nb % elem_size)
    return out


def gen_requests(rate_hz: float, duration_s: float, pool_sizes: list[int], seed: int = 5,
                 p_decompress: float = 0.6) -> list[Request]:
    """Poisson arrivals at rate_hz for duration_s; each request names a
    payload of the pool uniformly at random (so sizes follow the pool's
    log-uniform law) and is a decompression with probability p_decompress."""
    rng = _rng(seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        op = "decompress" if rng.random() < p_decompress else "compress"
        k = int(rng.integers(0, len(pool_sizes)))
        out.append(Request(len(out), t, op, k, pool_sizes[k]))
    return out
