"""The compress entry point that allocates nothing (its scratch space is the
library's fixed per-GPU array): called through the C-ABI, its streams equal
those of bsg_compress_lz4 with a caller workspace, byte for byte, on two
calls in a row, the second with a smaller input (so the array still holds
the first call's contents), and equal the oracle's."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1503_00638_amd import _lib, synth

pytestmark = pytest.mark.gpu


def _case(F, I, T, seed, cut):
    """Rounded CHIME-shaped visibilities as float32 elements, the last `cut`
    elements dropped (a partial block and a raw tail)."""
    vis, autos = synth.gen_vis(F, I, T, seed, 3.9e6)
    r = oracle.round_to_noise(vis, autos, 3.9e6, 0.01)
    flat = r.view(np.uint8).reshape(-1)
    return np.ascontiguousarray(flat[: flat.size - 4 * cut])


def _noalloc(L, torch, x, E, B, stream):
    n = x.numel() // E
    cap = L.bsg_compress_bound(n, E, B)
    out = torch.full((cap,), 0xAB, dtype=torch.uint8, device=x.device)
    nb = torch.zeros(1, dtype=torch.int64, device=x.device)
    rc = L.bsg_compress_lz4_noalloc(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    n, E, B, cap, ctypes.c_void_p(nb.data_ptr()),
                                    ctypes.c_void_p(stream.cuda_stream))
    assert rc == 0, rc
    return out, nb


def _with_workspace(L, torch, x, E, B, stream):
    n = x.numel() // E
    cap = L.bsg_compress_bound(n, E, B)
    out = torch.zeros(cap, dtype=torch.uint8, device=x.device)
    nb = torch.zeros(1, dtype=torch.int64, device=x.device)
    wsb = L.bsg_compress_workspace_size(n, E, B)
    ws = torch.empty(wsb, dtype=torch.uint8, device=x.device)
    rc = L.bsg_compress_lz4(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), n, E, B,
                            cap, ctypes.c_void_p(nb.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                            wsb, ctypes.c_void_p(stream.cuda_stream))
    assert rc == 0, rc
    return out, nb


def test_noalloc_equals_workspace_path_twice():
    import torch
    L = _lib.lib()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    # a 4.9 MB chunk in 8 KiB blocks first, then a 0.4 MB one in 2 KiB blocks
    cases = [(_case(64, 24, 32, 11, 5), 4, 2048), (_case(12, 16, 32, 12, 3), 4, 512)]
    for k, (host, E, B) in enumerate(cases):
        print(f"noalloc call {k}: {host.size} bytes, E={E}, block {B}", flush=True)
        n = host.size // E
        assert L.bsg_compress_workspace_size(n, E, B) <= _lib.NOALLOC_SCRATCH_BYTES
        x = torch.from_numpy(host.copy()).to(dev)
        o1, n1 = _noalloc(L, torch, x, E, B, stream)
        o2, n2 = _with_workspace(L, torch, x, E, B, stream)
        torch.cuda.synchronize()
        m1, m2 = int(n1.item()), int(n2.item())
        assert m1 == m2 > 0, (m1, m2)
        got = o1[:m1].cpu().numpy()
        assert np.array_equal(got, o2[:m2].cpu().numpy())
        assert np.array_equal(got, oracle.compress(host.view(np.uint32), E, B))


def test_noalloc_refuses_oversized_input():
    L = _lib.lib()
    n = (_lib.NOALLOC_SCRATCH_BYTES // 4) + (1 << 20)
    vp = ctypes.c_void_p
    assert L.bsg_compress_lz4_noalloc(vp(4096), vp(8192), n, 4, 2048, 1 << 40, vp(16), None) == -2
