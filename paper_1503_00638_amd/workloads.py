"""Device-resident inputs for the batched workload: many independent chunks
of uneven sizes and element widths (Section 4.2 treats blocks, and so
chunks of blocks, as independent units).

Chunk c has a size log-uniform in 64 KiB..64 MiB and an element size drawn
from {2, 4, 8}; half hold noise-rounded visibilities (the visibility model
at 16 inputs, as many frequencies as the size needs, rounded with f = 0.01),
half int16 random walks.  Raw content comes from the seeded device
generators in synth; the rounding is this library's round_to_noise.
"""
from __future__ import annotations

import torch

from . import round_to_noise, synth

F_DEFAULT = 0.01


def chunk_input(spec: synth.ChunkSpec, device="cuda", n_samples: float = synth.N_SAMPLES_DEFAULT,
                f: float = F_DEFAULT) -> torch.Tensor:
    """The chunk's bytes (device uint8, exactly spec.nbytes)."""
    if spec.kind == "walk":
        return synth.gen_walk_chunk_device(spec, device)
    vis, autos = synth.gen_chunk_vis_device(spec, device=device)
    round_to_noise(vis, autos, n_samples, f, out=vis)
    return vis.view(torch.uint8).reshape(-1)[: spec.nbytes]


def make_batch(count: int = 4096, seed: int = 3, device="cuda", lo: int = 1 << 16,
               hi: int = 1 << 26):
    """(specs, inputs) for the batched workload."""
    specs = synth.gen_batch_specs(count, seed, lo, hi)
    inputs = [chunk_input(s, device) for s in specs]
    return specs, inputs


# ---------------------------------------------------------------------------
# payload pool of the request stream
# ---------------------------------------------------------------------------
POOL_INPUTS, POOL_T, POOL_BLOCK_ELEMS = 128, 32, 2048  # CHIME-Pathfinder shape, 8 KiB blocks


class PoolEntry:
    """One device-resident payload: noise-rounded visibilities viewed as
    float32 elements, and its compressed stream."""

    def __init__(self, seed, data, stream, stream_len):
        self.seed, self.data, self.stream, self.stream_len = seed, data, stream, stream_len

    @property
    def nbytes(self) -> int:
        return self.data.numel()

    @property
    def n(self) -> int:
        return self.data.numel() // 4


def pool_raw_vis(size: int, seed: int, device="cuda"):
    """Raw (vis, autos) covering at least `size` bytes, config-1 shape."""
    per_f = synth.n_products(POOL_INPUTS) * POOL_T * 8
    F = max(1, -(-size // per_f))
    return synth.gen_vis_device(F, POOL_INPUTS, POOL_T, seed, device=device)


def make_pool(sizes, seed: int = 40, device="cuda", n_samples: float = synth.N_SAMPLES_DEFAULT,
              f: float = F_DEFAULT) -> list[PoolEntry]:
    from . import compress
    pool = []
    for k, size in enumerate(sizes):
        vis, autos = pool_raw_vis(size, seed + k, device)
        round_to_noise(vis, autos, n_samples, f, out=vis)
        data = vis.view(torch.uint8).reshape(-1)[:size].clone()
        del vis, autos
        out, nb = compress(data, 4, POOL_BLOCK_ELEMS)
        m = int(nb.item())
        pool.append(PoolEntry(seed + k, data, out[:m].clone(), m))
    return pool
