"""The C-ABI library: it loads on the CPU and exports every symbol the
header declares; host-only calls (sizes, header parsing, argument checks
that need no device) behave as documented.  No device work here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bsg.h")


def declared_symbols():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(bsg_[a-z0-9_]+)\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_1503_00638_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1503_00638_amd import build
        build.build()
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    syms = declared_symbols()
    assert "bsg_compress_lz4" in syms and "bsg_round_to_noise" in syms
    for s in syms:
        assert hasattr(L, s), s
    from paper_1503_00638_amd import _lib
    assert set(_lib.EXPORTS) == set(syms)


def test_host_only_calls(L):
    import oracle
    for E, B in ((4, 0), (4, 2048), (2, 4096), (1, 8192), (8, 1024), (16, 512), (3, 64)):
        for n in (0, 1, 7, 8, 12345, 2048 * 5 + 17):
            assert L.bsg_compress_bound(n, E, B) == oracle.compress_bound(n, E, B)
            assert L.bsg_block_elems(E, B) == oracle.block_elems(E, B)
            assert L.bsg_compress_workspace_size(n, E, B) > 0
    assert L.bsg_block_elems(0, 8) == -1
    assert L.bsg_block_elems(4, 12) == -1
    assert L.bsg_compress_bound(100, 4, 65536) == -1  # 256 KiB blocks exceed 16-bit offsets
    assert L.bsg_strerror(-3) == b"corrupt or mismatched compressed stream"


def test_argument_checks_need_no_device(L):
    vp = ctypes.c_void_p
    # invalid sizes and parameters are refused before any device call
    assert L.bsg_bitshuffle(vp(16), vp(32), -1, 4, 0, None) == -1
    assert L.bsg_bitshuffle(vp(16), vp(32), 64, 4, 12, None) == -1
    assert L.bsg_bitshuffle(None, None, 64, 4, 0, None) == -1
    assert L.bsg_round_to_noise(vp(16), vp(16), vp(16), 1, 2, 3, None, 3.9e6, -1.0, None) == -1
    assert L.bsg_round_to_noise(vp(16), vp(16), vp(16), 1, 2, 3, None, 0.0, 0.01, None) == -1
    assert L.bsg_decompress_lz4(vp(16), 10, vp(16), 2048, 4, 0, vp(16), None) == -3
    assert L.bsg_compress_lz4(vp(16), vp(16), 2048, 4, 0, 1 << 20, vp(16), vp(256), 0, None) == -2


def test_noalloc_argument_checks(L):
    """The entry point that allocates nothing refuses, on the host, inputs
    whose scratch space would exceed its fixed array, and bad block sizes."""
    from paper_1503_00638_amd import _lib
    vp = ctypes.c_void_p
    big = _lib.NOALLOC_SCRATCH_BYTES // 4 + (1 << 20)  # float32 elements
    assert L.bsg_compress_workspace_size(big, 4, 2048) > _lib.NOALLOC_SCRATCH_BYTES
    assert L.bsg_compress_lz4_noalloc(vp(4096), vp(8192), big, 4, 2048, 1 << 40, vp(16), None) == -2
    assert L.bsg_compress_lz4_noalloc(vp(4096), vp(8192), 100, 4, 12, 1 << 20, vp(16), None) == -1
    assert L.bsg_compress_lz4_noalloc(vp(4096), vp(8192), 100, 4, 1 << 16, 1 << 20, vp(16), None) == -1
    fits = L.bsg_compress_workspace_size((60 << 20) // 4, 4, 2048)
    assert 0 < fits <= _lib.NOALLOC_SCRATCH_BYTES


def test_prod_map_validated_before_any_launch():
    """A product map with an entry outside [0, I) would make the kernels read
    the autos out of bounds; the binding refuses it (host tensors here, so no
    device work is involved)."""
    import torch
    import paper_1503_00638_amd as bsg
    I, P = 4, 10
    ok = torch.tensor([[i, j] for i in range(I) for j in range(i, I)], dtype=torch.int32)
    bsg._check_prod_map(ok, P, I)
    bsg._check_prod_map(None, P, I)
    for bad in ([[0, 4]], [[-1, 0]], [[0, 2**30]]):
        m = ok.clone()
        m[3] = torch.tensor(bad[0], dtype=torch.int32)
        with pytest.raises(ValueError, match="entries"):
            bsg._check_prod_map(m, P, I)
    with pytest.raises(ValueError, match="int32"):
        bsg._check_prod_map(ok.to(torch.int64), P, I)
    with pytest.raises(ValueError, match="int32"):
        bsg._check_prod_map(ok[:5], P, I)


def test_read_header(L):
    import numpy as np
    import oracle
    import paper_1503_00638_amd as bsg
    s = oracle.compress(np.arange(5000, dtype=np.int32), 4, 1024)
    h = bsg.read_header(s.tobytes())
    assert (h.magic, h.elem_size, h.n, h.block_elems, h.n_blocks) == (0x31475342, 4, 5000, 1024, 5)
    with pytest.raises(bsg.BsgError):
        bsg.read_header(b"\0" * 24)


def test_batch_table_host_calls(L):
    """Descriptor tables are built on the host: sizes, validation and the
    workspace bound need no device."""
    from paper_1503_00638_amd import _lib
    assert L.bsg_batch_table_bytes(-1) == -1
    t0, t3 = L.bsg_batch_table_bytes(0), L.bsg_batch_table_bytes(3)
    assert 0 < t0 < t3
    vp = ctypes.c_void_p
    rows = [(4, 2048, 10000), (2, 0, 77), (8, 8192, 8192 * 2 + 5)]
    arr = (_lib.Chunk * 3)(*[_lib.Chunk(vp(4096), 0, vp(8192), 1 << 20, n, e, b) for e, b, n in rows])
    buf = ctypes.create_string_buffer(t3)
    assert L.bsg_batch_build_table(arr, 3, buf, t3) == 0
    assert L.bsg_batch_build_table(arr, 3, buf, t3 - 1) == -1
    ws = L.bsg_batch_workspace_size(buf)
    # workspace holds at least one bound-sized slot per block
    import oracle
    nblocks = sum((n // oracle.block_elems(e, b)) + 1 for e, b, n in rows)
    assert ws >= sum(oracle.compress_bound(n, e, b) for e, b, n in rows) - 32 * 3
    assert ws >= 4 * nblocks
    bad = (_lib.Chunk * 1)(_lib.Chunk(vp(4096), 0, vp(8192), 1 << 20, 100, 4, 12))  # block % 8
    assert L.bsg_batch_build_table(bad, 1, buf, t3) == -1
    big = (_lib.Chunk * 1)(_lib.Chunk(vp(4096), 0, vp(8192), 1 << 20, 100, 8, 16384))  # 128 KiB
    assert L.bsg_batch_build_table(big, 1, buf, t3) == -1
    assert L.bsg_batch_compress(buf, None, vp(256), vp(256), 1 << 20, 0, 0, None) == -1
    assert L.bsg_batch_decompress(buf, vp(17), vp(256), 0, 0, None) == -1
    # an unknown block schedule is refused before any device work
    assert L.bsg_batch_compress(buf, vp(4096), vp(256), vp(256), 1 << 30, 0, 2, None) == -1
    assert L.bsg_batch_decompress(buf, vp(4096), vp(256), 0, -1, None) == -1


def _gfx950_kernel_metadata(lib_path, tmp_path):
    """(kernel name, private segment bytes per lane) of every kernel in the
    library's gfx950 code objects (one offload bundle per source file)."""
    import shutil
    import subprocess
    llvm = "/opt/rocm/llvm/bin"
    tools = [shutil.which("objcopy"), os.path.join(llvm, "clang-offload-bundler"),
             os.path.join(llvm, "llvm-readelf")]
    if tools[0] is None or not all(os.path.exists(t) for t in tools[1:]):
        pytest.skip("no objcopy / clang-offload-bundler / llvm-readelf")
    # objcopy rewrites the file it reads unless given an output file: work on
    # a copy, so the library this process has loaded is never touched
    lib_copy = tmp_path / "lib.so"
    shutil.copyfile(lib_path, lib_copy)
    fat = tmp_path / "fatbin.bin"
    subprocess.run([tools[0], "--dump-section", f".hip_fatbin={fat}", str(lib_copy),
                    str(tmp_path / "lib_out.so")], check=True)
    data = fat.read_bytes()
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    starts = [m.start() for m in re.finditer(re.escape(magic), data)] + [len(data)]
    out = []
    for k in range(len(starts) - 1):
        b = tmp_path / f"b{k}.bin"
        co = tmp_path / f"c{k}.co"
        b.write_bytes(data[starts[k]:starts[k + 1]])
        subprocess.run([tools[1], "--unbundle", "--type=o", f"--input={b}",
                        "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"], check=True)
        notes = subprocess.run([tools[2], "--notes", str(co)], capture_output=True, text=True,
                               check=True).stdout.splitlines()
        names = [l.split(":", 1)[1].strip() for l in notes if l.strip().startswith(".name:")]
        sizes = [int(l.split(":", 1)[1]) for l in notes if "private_segment_fixed_size" in l]
        assert len(names) == len(sizes)
        out += list(zip(names, sizes))
    return out


def test_kernels_use_no_scratch(L, tmp_path):
    """No kernel spills to scratch (per-lane private memory in HBM): every
    kernel's private segment is empty."""
    from paper_1503_00638_amd import _lib
    meta = _gfx950_kernel_metadata(_lib.LIB_PATH, tmp_path)
    assert any("k_encode" in n for n, _ in meta) and any("k_decode" in n for n, _ in meta)
    spill = [(n, s) for n, s in meta if s != 0]
    assert not spill, spill
