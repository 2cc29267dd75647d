"""GPU parity: every HIP output equals the CPU oracle bit for bit.

Inputs are seeded synthetic stand-ins for the paper's workloads (see
paper_1503_00638_amd/synth.py); the oracle is oracle/ (plain C).  Sizes here
are small enough for the oracle to finish in seconds while spanning several
blocks/tiles and ragged tails; the full-size workloads are in
test_gpu_full.py."""
import numpy as np
import pytest

import lz4ref
import oracle
from paper_1503_00638_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 3.9e6


@pytest.fixture(scope="module")
def bsg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1503_00638_amd as m
    m.load()
    return m


def dev(a):
    return torch.from_numpy(np.array(a, copy=True, order="C")).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def u32(a):
    return np.ascontiguousarray(a).view(np.uint32)


# ---------------------------------------------------------------- rounding
@pytest.mark.parametrize("F,I,T,seed,f", [(16, 8, 64, 0, 0.01), (3, 5, 7, 1, 0.01), (1, 1, 1, 2, 0.1),
                                          (2, 16, 33, 3, 1e-3), (4, 12, 5, 4, 1e-5), (2, 3, 9, 5, 0.0)])
def test_round_parity(bsg, F, I, T, seed, f):
    vis, autos = synth.gen_vis(F, I, T, seed, N)
    ref = oracle.round_to_noise(vis, autos, N, f)
    got = host(bsg.round_to_noise(dev(vis), dev(autos), N, f))
    assert np.array_equal(u32(got), u32(ref))


def test_round_special_values(bsg):
    rng = np.random.default_rng(9)
    F, I, T = 3, 6, 40
    vis, autos = synth.gen_vis(F, I, T, 9, N)
    vf = vis.view(np.float32).reshape(-1)
    bits = rng.integers(0, 2 ** 32, vf.size // 2, dtype=np.uint64).astype(np.uint32)
    vf[::2] = bits.view(np.float32)  # every float class: NaN, Inf, subnormal, huge
    vf[1::7] = np.float32(0.0)
    vf[3::11] = np.float32(-0.0)
    autos[0, 0, :5] = [0.0, -1.0, np.nan, np.inf, 1e-40]
    autos[1, 2, :4] = [3.4e38, 1e-30, 1e30, 1e-45]
    autos[2] *= np.float32(2.0 ** 60)
    for f in (0.01, 1e-5, 7.0):
        ref = oracle.round_to_noise(vis, autos, N, f)
        got = host(bsg.round_to_noise(dev(vis), dev(autos), N, f))
        assert np.array_equal(u32(got), u32(ref)), f
        # the same rounding fused into the encoder's staging: 2048-element
        # blocks take the 16-visibility register path where a unit stays in
        # one product, the per-visibility path where it crosses one, and the
        # ragged last block the generic path
        fused, nb = bsg.round_compress(dev(vis), dev(autos), N, f, block_size=2048)
        m = int(host(nb)[0])
        assert np.array_equal(host(fused)[:m], oracle.compress(ref, 4, 2048)), f


def ties_at_binade_inputs():
    """Crafted rounding cases where g equals the power of two at the start of
    x's binade (x in [g, 2g)), including the exact tie x = 1.5 g, for even and
    odd biased exponents.  With f = 1 and N = 6 the cross G2 is V_ii V_jj, and
    V = 1.5 * 2^K gives k = K."""
    Ks = list(range(-20, 21))
    T = len(Ks)
    autos = np.empty((1, 2, T), dtype=np.float32)
    autos[0, 0] = [1.5 * 2.0 ** K for K in Ks]
    autos[0, 1] = autos[0, 0]
    vis = np.zeros((1, 3, T), dtype=np.complex64)
    mult = [1.5, 1.25, 1.75, 1.5 + 2 ** -20, 1.5 - 2 ** -20, -1.5, 1.0, 2.0 - 2 ** -22]
    out = []
    for m in mult:
        v = vis.copy()
        for t, K in enumerate(Ks):
            g = 2.0 ** K
            v[0, 1, t] = np.complex64(complex(m * g, -m * g * 0.5))
            v[0, 0, t] = np.complex64(complex(m * g * 1.5, m * g))
            v[0, 2, t] = np.complex64(complex(-m * g, m * g))
        out.append(v)
    return out, autos


def test_round_ties_at_binade(bsg):
    vs, autos = ties_at_binade_inputs()
    for v in vs:
        ref = oracle.round_to_noise(v, autos, 6.0, 1.0)
        got = host(bsg.round_to_noise(dev(v), dev(autos), 6.0, 1.0))
        assert np.array_equal(u32(got), u32(ref))
        fused, nb = bsg.round_compress(dev(v), dev(autos), 6.0, 1.0, block_size=8)
        m = int(host(nb)[0])
        assert np.array_equal(host(fused)[:m], oracle.compress(ref, 4, 8))


def test_round_prod_map_and_in_place(bsg):
    F, I, T = 2, 7, 16
    vis, autos = synth.gen_vis(F, I, T, 11, N)
    pairs = synth.product_pairs(I)
    perm = np.random.default_rng(1).permutation(len(pairs))
    pm = np.ascontiguousarray(pairs[perm])
    v2 = np.ascontiguousarray(vis[:, perm])
    ref = oracle.round_to_noise(v2, autos, N, 0.01, prod_map=pm)
    d = dev(v2)
    bsg.round_to_noise(d, dev(autos), N, 0.01, out=d, prod_map=dev(pm))
    assert np.array_equal(u32(host(d)), u32(ref))


# ---------------------------------------------------------------- transpose
SHUF_CASES = [(4, 2048, 2048 * 9), (4, 2048, 2048 * 3 + 8 * 37 + 5), (1, 8192, 8192 * 2 + 13),
              (2, 4096, 4096 * 2 + 8 * 3 + 1), (8, 1024, 1024 * 5 + 7), (16, 512, 512 * 4 + 40),
              (12, 64, 64 * 7 + 24), (3, 2728, 10000), (5, 16, 999), (4, 16, 1000),
              (1, 8, 64), (2, 64, 63), (4, 65536 // 4, 65536 // 4 * 2 + 100), (4, 0, 5000),
              (7, 24, 24 * 5), (16, 8, 100), (4, 40, 4000), (1, 136, 136 * 9 + 72)]


@pytest.mark.parametrize("E,nb,n", SHUF_CASES)
def test_bitshuffle_parity(bsg, E, nb, n):
    rng = np.random.default_rng(E * 7 + n)
    data = rng.integers(0, 256, n * E, dtype=np.uint8)
    ref = oracle.bitshuffle(data, E, nb)
    got = host(bsg.bitshuffle(dev(data), E, nb))
    assert np.array_equal(got, ref)
    back = host(bsg.bitunshuffle(dev(ref), E, nb))
    assert np.array_equal(back, data)


def test_bitshuffle_unaligned_pointers(bsg):
    rng = np.random.default_rng(3)
    E, nb, n = 4, 2048, 2048 * 3 + 24
    raw = dev(rng.integers(0, 256, n * E + 8, dtype=np.uint8))
    x = raw[4:4 + n * E]
    ref = oracle.bitshuffle(host(x), E, nb)
    out = torch.empty(n * E + 4, dtype=torch.uint8, device="cuda:0")
    got = bsg.bitshuffle(x, E, nb, out=out[4:])
    assert np.array_equal(host(got), ref)


@pytest.mark.parametrize("k", [4, 12, 20])
def test_bitshuffle_gauss_int32(bsg, k):
    x = synth.gen_gauss_int32(2048 * 16 + 8 * 5, k, k)
    for E in (1, 2, 4, 8):
        ref = oracle.bitshuffle(x, E, 8192 // E)
        got = host(bsg.bitshuffle(dev(x), E, 8192 // E))
        assert np.array_equal(got, ref), E


# ---------------------------------------------------------------- LZ4 streams
STREAM_CASES = [(4, 2048, 2048 * 6), (4, 2048, 2048 * 6 + 8 * 11 + 3), (2, 4096, 4096 * 3 + 1000),
                (8, 1024, 1024 * 4 + 9), (1, 8192, 8192 * 3 + 7), (16, 512, 512 * 3 + 16),
                (3, 64, 999), (4, 16, 1), (4, 16, 0), (4, 8, 64), (12, 512, 2000),
                (4, 16384, 16384 * 2 + 100), (2, 32768, 32768 + 8)]


def stream_inputs(E, n, seed):
    rng = np.random.default_rng(seed)
    kinds = [
        rng.integers(0, 256, n * E, dtype=np.uint8),  # incompressible
        (rng.integers(0, 4, n * E, dtype=np.uint8) * 17).astype(np.uint8),
        np.zeros(n * E, np.uint8),
        np.resize(rng.integers(0, 256, 300, dtype=np.uint8), n * E),
        synth.gen_walk_int16(n * E // 2 + 1, seed).view(np.uint8)[: n * E].copy(),
    ]
    return kinds


@pytest.mark.parametrize("E,nb,n", STREAM_CASES)
def test_compress_parity(bsg, E, nb, n):
    for data in stream_inputs(E, n, E * 31 + n):
        ref = oracle.compress(data, E, nb)
        x = dev(data) if data.size else torch.empty(0, dtype=torch.uint8, device="cuda:0")
        got = host(bsg.compress_sync(x, E, nb))
        assert got.size == ref.size and np.array_equal(got, ref)
        back = host(bsg.decompress_sync(dev(ref), n, E, nb))
        assert np.array_equal(back[: n * E], data)


def _lz4_sequence_count(block: bytes) -> int:
    """Sequences in one LZ4 block (token walk only)."""
    ip, n = 0, 0
    while ip < len(block):
        tok = block[ip]
        ip += 1
        ll = tok >> 4
        if ll == 15:
            while True:
                ip += 1
                ll += block[ip - 1]
                if block[ip - 1] != 255:
                    break
        ip += ll
        n += 1
        if ip >= len(block):
            break
        ip += 2
        if tok & 15 == 15:
            while block[ip] == 255:
                ip += 1
            ip += 1
    return n


@pytest.mark.parametrize("E,nb", [(4, 2048), (1, 8192), (2, 4096)])
def test_compress_many_sequences(bsg, E, nb):
    """Blocks that parse into ~500 short sequences, so the encoder writes
    them in several batches of 64 per block: the transposed domain holds an
    LZ77-like source of short matches (synth.gen_short_matches), the input
    is its inverse bit transpose."""
    P = synth.gen_short_matches(nb * E * 3 + 500, 11 + E)
    n = P.size // E
    data = oracle.bitunshuffle(P[: n * E], E, nb)
    ref = oracle.compress(data, E, nb)
    nblk = int(np.frombuffer(ref[20:24].tobytes(), dtype="<u4")[0])
    offs = np.frombuffer(ref[24:24 + 8 * (nblk + 1)].tobytes(), dtype="<u8")
    pay = ref[24 + 8 * (nblk + 1):].tobytes()
    counts = [_lz4_sequence_count(pay[offs[i]:offs[i + 1]]) for i in range(nblk)]
    assert max(counts) > 3 * 64, counts
    got = host(bsg.compress_sync(dev(data), E, nb))
    assert got.size == ref.size and np.array_equal(got, ref)
    back = host(bsg.decompress_sync(dev(ref), n, E, nb))
    assert np.array_equal(back[: n * E], data)


def _segmented_input():
    # 50,000 blocks of 512 bytes plus a ragged end: three segments of at
    # least 16,384 blocks, so the encoder runs in segments on two streams
    # and a third stream packs each finished segment
    E, nb = 4, 128
    x = np.concatenate([synth.gen_gauss_int32(nb * 24000, 7, 31),
                        synth.gen_gauss_int32(nb * 26000 + 45, 2, 32)]).view(np.uint8)
    return x, E, nb


def test_compress_segmented(bsg):
    """A large input compressed in segments: the stream equals the oracle's;
    with too little room the call reports the capacity error and writes
    nothing past the capacity it was given."""
    x, E, nb = _segmented_input()
    ref = oracle.compress(x, E, nb)
    got = host(bsg.compress_sync(dev(x), E, nb))
    assert got.size == ref.size and np.array_equal(got, ref)
    for cap in (ref.size - 1, ref.size // 2):
        big = torch.full((ref.size + 4096,), 0xA5, dtype=torch.uint8, device="cuda:0")
        _, st = bsg.compress(dev(x), E, nb, out=big[:cap])
        assert int(host(st)[0]) == -2
        assert bool((big[cap:] == 0xA5).all())


def test_compress_segmented_in_a_graph(bsg):
    """The segmented compression (which forks onto the library's own streams
    and joins back) captured in a graph and replayed three times, with
    other work and synchronisations between the replays: every replay's
    stream equals the eager one."""
    x, E, nb = _segmented_input()
    xd = dev(x)
    out, nbytes = bsg.compress(xd, E, nb)
    torch.cuda.synchronize()
    m = int(nbytes.item())
    eager = out[:m].clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        out2 = torch.empty_like(out)
        ws = torch.empty(bsg.workspace_size(x.size // E, E, nb), dtype=torch.uint8, device="cuda:0")
        nb2 = torch.empty(1, dtype=torch.int64, device="cuda:0")
        bsg.compress(xd, E, nb, out=out2, workspace=ws, nbytes=nb2, stream=s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        bsg.compress(xd, E, nb, out=out2, workspace=ws, nbytes=nb2, stream=s)
    for k in range(3):
        out2.fill_(k)
        nb2.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(nb2.item()) == m, k
        assert torch.equal(out2[:m], eager), k
        _ = (xd[:4096].float() * 2).sum().item()  # eager work between replays


def test_pipeline_config0(bsg):
    """Tiny plain pipeline: (16, 36, 64) complex64, f = 0.01, 8 KiB blocks."""
    vis, autos = synth.gen_vis(16, 8, 64, 0, N)
    r = oracle.round_to_noise(vis, autos, N, 0.01)
    ref = oracle.compress(r, 4, 2048)
    dr = bsg.round_to_noise(dev(vis), dev(autos), N, 0.01)
    s = bsg.compress_sync(dr.view(torch.uint8).reshape(-1), 4, 2048)
    assert np.array_equal(host(s), ref)
    fused, nb = bsg.round_compress(dev(vis), dev(autos), N, 0.01, block_size=2048)
    m = int(host(nb)[0])
    assert np.array_equal(host(fused)[:m], ref)
    d = bsg.decompress_sync(s, r.size * 2, 4, 2048)
    assert np.array_equal(host(d), r.view(np.uint8).reshape(-1))


@pytest.mark.parametrize("F,I,T,B", [(3, 5, 7, 2048), (2, 16, 33, 512), (5, 4, 3, 40), (1, 2, 1, 8),
                                     (4, 8, 64, 0)])
def test_fused_round_compress(bsg, F, I, T, B):
    vis, autos = synth.gen_vis(F, I, T, F * I + T, N)
    for f in (0.01, 0.0, 1e-4):
        r = oracle.round_to_noise(vis, autos, N, f)
        ref = oracle.compress(r, 4, B)
        out, nb = bsg.round_compress(dev(vis), dev(autos), N, f, block_size=B)
        m = int(host(nb)[0])
        assert m == ref.size and np.array_equal(host(out)[:m], ref), f


def test_decode_liblz4_payloads(bsg):
    """Streams whose blocks were encoded by the system liblz4 (greedy and HC):
    the decoder must accept any valid LZ4 block, not only its own."""
    if not lz4ref.available():
        pytest.skip("no liblz4")
    E, nb = 4, 2048
    vis, autos = synth.gen_vis(4, 8, 64, 7, N)
    r = oracle.round_to_noise(vis, autos, N, 0.01)
    sh = oracle.bitshuffle(r, E, nb)
    n = r.size * 2
    full, rem = divmod(n, nb)
    blocks = [sh[b * nb * E:(b + 1) * nb * E].tobytes() for b in range(full)]
    blocks.append(bytes(nb * E))
    blocks.append(bytes(range(256)) * (nb * E // 256))
    data_sh = b"".join(blocks)
    nblk = len(blocks)
    for enc in (lz4ref.compress_default, lz4ref.compress_hc):
        pays = [enc(b) for b in blocks]
        off = np.zeros(nblk + 1, dtype=np.uint64)
        off[1:] = np.cumsum([len(p) for p in pays])
        hdr = np.array([0x31475342, E], dtype=np.uint32).tobytes() + \
            np.array([nblk * nb], dtype=np.uint64).tobytes() + \
            np.array([nb, nblk], dtype=np.uint32).tobytes()
        stream = np.frombuffer(hdr + off.tobytes() + b"".join(pays), dtype=np.uint8)
        expect = oracle.bitunshuffle(np.frombuffer(data_sh, np.uint8), E, nb)
        got = host(bsg.decompress_sync(dev(stream), nblk * nb, E, nb))
        assert np.array_equal(got, expect)


def test_decode_overlapping_periods(bsg):
    """Overlapping matches of every small period: blocks holding a random
    pattern of period 1..20 after 0..3 random bytes, encoded by the system
    liblz4, so the decoder replicates periods shorter and longer than a
    dword at every byte phase."""
    if not lz4ref.available():
        pytest.skip("no liblz4")
    E, nb = 4, 2048
    rng = np.random.default_rng(21)
    blocks = []
    for p in range(1, 21):
        lead = p % 4
        pat = rng.integers(0, 256, p, dtype=np.uint8)
        body = np.resize(pat, nb * E - lead)
        blocks.append(rng.integers(0, 256, lead, dtype=np.uint8).tobytes() + body.tobytes())
    nblk = len(blocks)
    data_sh = b"".join(blocks)
    for enc in (lz4ref.compress_default, lz4ref.compress_hc):
        pays = [enc(b) for b in blocks]
        off = np.zeros(nblk + 1, dtype=np.uint64)
        off[1:] = np.cumsum([len(q) for q in pays])
        hdr = np.array([0x31475342, E], dtype=np.uint32).tobytes() + \
            np.array([nblk * nb], dtype=np.uint64).tobytes() + \
            np.array([nb, nblk], dtype=np.uint32).tobytes()
        stream = np.frombuffer(hdr + off.tobytes() + b"".join(pays), dtype=np.uint8)
        expect = oracle.bitunshuffle(np.frombuffer(data_sh, np.uint8), E, nb)
        got = host(bsg.decompress_sync(dev(stream), nblk * nb, E, nb))
        assert np.array_equal(got, expect)


def test_decode_long_overlapping_periods(bsg):
    """Overlapping matches with long periods in 64 KiB blocks (offsets up to
    40000, every byte phase of the period start), encoded by the oracle and,
    when present, by the system liblz4: the decoder's per-lane position in
    the period and its advance per step are exact for large offsets."""
    E, nb = 4, 16384
    rng = np.random.default_rng(22)
    periods = [21, 63, 64, 65, 255, 256, 257, 1021, 4093, 8192, 8193, 20000, 32767, 40000]
    blocks = []
    for k, p in enumerate(periods):
        lead = k % 4
        pat = rng.integers(0, 256, p, dtype=np.uint8)
        body = np.resize(pat, nb * E - lead)
        blocks.append(rng.integers(0, 256, lead, dtype=np.uint8).tobytes() + body.tobytes())
    nblk = len(blocks)
    data_sh = b"".join(blocks)
    expect = oracle.bitunshuffle(np.frombuffer(data_sh, np.uint8), E, nb)
    encoders = [lambda b: oracle.lz4_compress_block(np.frombuffer(b, np.uint8))]
    if lz4ref.available():
        encoders += [lz4ref.compress_default, lz4ref.compress_hc]
    for enc in encoders:
        pays = [enc(b) for b in blocks]
        off = np.zeros(nblk + 1, dtype=np.uint64)
        off[1:] = np.cumsum([len(q) for q in pays])
        hdr = np.array([0x31475342, E], dtype=np.uint32).tobytes() + \
            np.array([nblk * nb], dtype=np.uint64).tobytes() + \
            np.array([nb, nblk], dtype=np.uint32).tobytes()
        stream = np.frombuffer(hdr + off.tobytes() + b"".join(pays), dtype=np.uint8)
        got = host(bsg.decompress_sync(dev(stream), nblk * nb, E, nb))
        assert np.array_equal(got, expect)


def test_decode_offsets_from_256_in_8k_blocks(bsg):
    """Overlapping matches at offsets on both sides of 256 bytes (the output
    of one 64-lane copy step) in the 8 KiB blocks of the hot path, every
    byte phase of the period start, some periods broken by a changed byte,
    encoded by the oracle and, when present, by the system liblz4."""
    E, nb = 4, 2048
    rng = np.random.default_rng(23)
    periods = [255, 256, 257, 258, 259, 300, 511, 512, 513, 1024, 2047, 4096]
    blocks = []
    for k, p in enumerate(periods):
        lead = k % 4
        pat = rng.integers(0, 256, p, dtype=np.uint8)
        body = np.resize(pat, nb * E - lead)
        if k % 3 == 2:  # a changed byte ends one match and starts another
            body[int(rng.integers(p, body.size))] ^= 0x5A
        blocks.append(rng.integers(0, 256, lead, dtype=np.uint8).tobytes() + body.tobytes())
    nblk = len(blocks)
    data_sh = b"".join(blocks)
    expect = oracle.bitunshuffle(np.frombuffer(data_sh, np.uint8), E, nb)
    encoders = [lambda b: oracle.lz4_compress_block(np.frombuffer(b, np.uint8))]
    if lz4ref.available():
        encoders += [lz4ref.compress_default, lz4ref.compress_hc]
    for enc in encoders:
        pays = [enc(b) for b in blocks]
        assert any(q[1] is not None and q[1] >= 256 and q[2] > q[1]
                   for pay in pays for q in lz4ref.parse_sequences(pay))
        off = np.zeros(nblk + 1, dtype=np.uint64)
        off[1:] = np.cumsum([len(q) for q in pays])
        hdr = np.array([0x31475342, E], dtype=np.uint32).tobytes() + \
            np.array([nblk * nb], dtype=np.uint64).tobytes() + \
            np.array([nb, nblk], dtype=np.uint32).tobytes()
        stream = np.frombuffer(hdr + off.tobytes() + b"".join(pays), dtype=np.uint8)
        got = host(bsg.decompress_sync(dev(stream), nblk * nb, E, nb))
        assert np.array_equal(got, expect)


def test_decode_rejects_corruption(bsg):
    E, nb = 4, 2048
    x = synth.gen_gauss_int32(2048 * 8 + 5, 6, 2)
    s = oracle.compress(x, E, nb)
    rng = np.random.default_rng(4)
    table_end = 24 + 8 * 9
    n_err = 0
    for trial in range(60):
        c = s.copy()
        kind = trial % 4
        if kind == 0:
            i = int(rng.integers(table_end, c.size))
            c[i] ^= np.uint8(1 << int(rng.integers(0, 8)))
            nbytes = c.size
        elif kind == 1:  # offset table entry
            i = int(rng.integers(24, table_end))
            c[i] ^= np.uint8(1 << int(rng.integers(0, 8)))
            nbytes = c.size
        elif kind == 2:  # header field
            i = int(rng.integers(0, 24))
            c[i] ^= np.uint8(1 << int(rng.integers(0, 8)))
            nbytes = c.size
        else:  # stream shorter than it claims
            nbytes = int(rng.integers(table_end + 28, c.size))
        out, st = bsg.decompress(dev(c), nbytes, x.size, E, nb)
        code = int(host(st)[0])
        try:
            ref = oracle.decompress(c[:nbytes], x.size, E, nb)
            ref_ok = True
        except oracle.OracleError:
            ref_ok = False
        assert (code == 0) == ref_ok, (trial, code)
        if ref_ok:
            assert np.array_equal(host(out)[: x.size * 4], ref)
        else:
            assert code == -3
            n_err += 1
    assert n_err > 20


def test_compress_near_uniform_groups(bsg):
    """Blocks whose LZ4 input (the transposed block) is one byte value except
    for a single byte at the edges of a 512-position hash group (the group's
    last window reaches 3 bytes into the next one), and blocks whose value
    changes exactly at group boundaries: the stream equals the oracle's and
    decodes back."""
    E, nb = 4, 2048
    n = nb * E
    blocks = []
    for g0 in (0, 1536, 7168):
        for k in (0, 1, 63, 64, 65, 511, 512, 513, 514, 515):
            if g0 + k < n:
                t = np.full(n, 0x33, dtype=np.uint8)
                t[g0 + k] = 0x5A
                blocks.append(t)
    t = np.repeat(np.arange(16, dtype=np.uint8) * 17, 512)
    blocks.append(t)
    t = t.copy()
    t[512 * 3 - 1] = 0
    blocks.append(t)
    blocks.append(np.zeros(n, dtype=np.uint8))
    trans = np.concatenate(blocks)
    data = oracle.bitunshuffle(trans, E, nb)
    ref = oracle.compress(data, E, nb)
    got = host(bsg.compress_sync(dev(data), E, nb))
    assert np.array_equal(got, ref)
    back = host(bsg.decompress_sync(dev(ref), data.size // E, E, nb))
    assert np.array_equal(back, data)


def _lz4_len(n):
    """LZ4 length continuation bytes for a length field value n >= 15."""
    out, r = [], n - 15
    while r >= 255:
        out.append(255)
        r -= 255
    return out + [r]


def test_decode_rejects_overlong_literals(bsg):
    """Blocks whose literal runs end past the block (as the last sequence,
    or before a match), whose match offset is 0 or reaches before the
    block's start, and a block with no bytes at all are rejected, as by the
    oracle, and the blocks around them still decode."""
    E, nb = 4, 2048
    n = nb * E
    rng = np.random.default_rng(23)
    lit = rng.integers(0, 256, n + 64, dtype=np.uint8).tobytes()
    good = oracle.lz4_compress_block(np.frombuffer(lit[:n], np.uint8))

    def seq(ll, body, off=None, ml=None):
        tok = (min(ll, 15) << 4) | (0 if ml is None else min(ml - 4, 15))
        b = bytes([tok] + (_lz4_len(ll) if ll >= 15 else [])) + body[:ll]
        if ml is not None:
            b += bytes([off & 255, off >> 8]) + bytes(_lz4_len(ml - 4) if ml - 4 >= 15 else [])
        return b

    bad_blocks = [
        seq(n + 5, lit),                                  # last literals past the block
        seq(n - 2, lit, off=1, ml=10) + seq(0, b""),      # match past the block
        seq(n + 3, lit, off=1, ml=4) + seq(0, b""),       # literals past it, then a match
        b"",                                              # no token at all
        seq(8, lit, off=0, ml=4) + seq(0, b""),           # offset 0
        seq(8, lit, off=9, ml=4) + seq(0, b""),           # offset before the block start
        seq(8, lit, off=8, ml=n - 10) + seq(5, lit),      # next literals end past the block
    ]
    for bad in bad_blocks:
        with pytest.raises(oracle.OracleError):
            oracle.lz4_decompress_block(bad, n)
        pays = [good, bad, good]
        off = np.zeros(4, dtype=np.uint64)
        off[1:] = np.cumsum([len(q) for q in pays])
        hdr = np.array([0x31475342, E], dtype=np.uint32).tobytes() + \
            np.array([3 * nb], dtype=np.uint64).tobytes() + \
            np.array([nb, 3], dtype=np.uint32).tobytes()
        stream = np.frombuffer(hdr + off.tobytes() + b"".join(pays), dtype=np.uint8)
        out, st = bsg.decompress(dev(stream), stream.size, 3 * nb, E, nb)
        assert int(host(st)[0]) == -3, len(bad)
        got = host(out)
        expect = oracle.bitunshuffle(np.frombuffer(lit[:n], np.uint8), E, nb)
        assert np.array_equal(got[:n], expect) and np.array_equal(got[2 * n:3 * n], expect)


def test_capacity_verdict(bsg):
    x = np.random.default_rng(0).integers(0, 256, 2048 * 4 * 4, dtype=np.uint8)
    ref = oracle.compress(x, 4, 2048)
    need = bsg.compress_bound(x.size // 4, 4, 2048)
    out = torch.empty(ref.size - 1, dtype=torch.uint8, device="cuda:0")
    _, nb = bsg.compress(dev(x), 4, 2048, out=out)
    assert int(host(nb)[0]) == -2
    out = torch.empty(ref.size, dtype=torch.uint8, device="cuda:0")
    _, nb = bsg.compress(dev(x), 4, 2048, out=out)
    assert int(host(nb)[0]) == ref.size <= need
    assert np.array_equal(host(out), ref)


def test_repeatable_and_stream_order(bsg):
    vis, autos = synth.gen_vis(8, 16, 32, 5, N)
    dv, da = dev(vis), dev(autos)
    outs = []
    s = torch.cuda.Stream()
    for k in range(3):
        with torch.cuda.stream(s if k == 1 else torch.cuda.current_stream()):
            o, nb = bsg.round_compress(dv, da, N, 0.01, block_size=2048, stream=s if k == 1 else None)
            torch.cuda.synchronize()
            outs.append(host(o)[: int(host(nb)[0])])
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


def test_compress_segmented_two_threads(bsg):
    """Two host threads compress large inputs at the same time, each on its
    own stream: the library's side streams and their events are shared and
    taken in turn, and both streams come out equal to the oracle's."""
    import threading
    x, E, nb = _segmented_input()
    y = x[::-1].copy()
    refs = [oracle.compress(x, E, nb), oracle.compress(y, E, nb)]
    xs = [dev(x), dev(y)]
    torch.cuda.synchronize()
    outs = [None, None]

    def work(k):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            for _ in range(3):
                o, m = bsg.compress(xs[k], E, nb, stream=s)
            s.synchronize()
            outs[k] = (o, m)

    th = [threading.Thread(target=work, args=(k,)) for k in (0, 1)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for k in (0, 1):
        o, m = outs[k]
        n = int(host(m)[0])
        assert n == refs[k].size and np.array_equal(host(o)[:n], refs[k]), k
