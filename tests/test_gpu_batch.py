"""GPU parity of the batch entry points: many independent chunks of mixed
element sizes, block sizes and lengths in one call.  Every chunk's stream
equals the oracle's stream for that chunk alone, byte for byte, and the batch
decoder restores every chunk; capacity and corruption verdicts are per
chunk; a captured CUDA graph of the batch replays to the same bytes."""
import numpy as np
import pytest

import oracle
from paper_1503_00638_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 3.9e6

# (elem_size, block elems, n): fast element classes 1/2/4/8/12/16 and the
# generic path (3, 6), 8 KiB and 64 KiB blocks, ragged tails, a block-exact
# chunk, one-element and empty chunks.
MIX = [(4, 2048, 2048 * 3 + 13), (2, 4096, 4096 * 2 + 8), (1, 8192, 8192 * 2 + 7),
       (8, 1024, 1024 * 5), (3, 64, 999), (16, 512, 512 * 3 + 16), (12, 512, 2000),
       (4, 16384, 16384 * 2 + 100), (2, 32768, 32768 + 8), (4, 16, 1), (4, 16, 0),
       (6, 256, 3000), (4, 2048, 2048), (8, 8192, 8192 + 3), (1, 65536, 65536 * 2 + 9)]


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


def chunk_data(k, E, n):
    rng = np.random.default_rng(100 + k)
    kind = k % 4
    if kind == 0:
        return rng.integers(0, 256, n * E, dtype=np.uint8)
    if kind == 1:
        return synth.gen_walk_int16(n * E // 2 + 1, k).view(np.uint8)[: n * E].copy()
    if kind == 2:
        return (rng.integers(0, 4, n * E, dtype=np.uint8) * 17).astype(np.uint8)
    return np.resize(rng.integers(0, 256, 300, dtype=np.uint8), n * E)


def mixed():
    data = [chunk_data(k, E, n) for k, (E, _, n) in enumerate(MIX)]
    # one chunk of rounded visibilities (float32 elements), as the pipeline makes
    vis, autos = synth.gen_vis(3, 8, 40, 11, N)
    data.append(oracle.round_to_noise(vis, autos, N, 0.01).view(np.uint8).reshape(-1))
    Es = [E for E, _, _ in MIX] + [4]
    Bs = [b for _, b, _ in MIX] + [2048]
    return data, Es, Bs


def to_dev(a):
    return dev(a) if a.size else torch.empty(0, dtype=torch.uint8, device="cuda:0")


def test_batch_compress_and_decompress_parity(bsg):
    data, Es, Bs = mixed()
    refs = [oracle.compress(d, E, B) for d, E, B in zip(data, Es, Bs)]
    xs = [to_dev(d) for d in data]
    plan = bsg.BatchPlan.for_compress(xs, Es, Bs)
    nb = host(plan.compress())
    for k, ref in enumerate(refs):
        assert nb[k] == ref.size, k
        assert np.array_equal(host(plan.outs[k])[: ref.size], ref), k
    ns = [d.size // E for d, E in zip(data, Es)]
    dplan = bsg.BatchPlan.for_decompress(plan.outs, nb.tolist(), ns, Es, Bs)
    st = host(dplan.decompress())
    assert not st.any(), st
    for k, d in enumerate(data):
        assert np.array_equal(host(dplan.outs[k])[: d.size], d), k


def test_batch_launch_shape_does_not_change_bytes(bsg):
    data, Es, Bs = mixed()
    xs = [to_dev(d) for d in data]
    plan = bsg.BatchPlan.for_compress(xs, Es, Bs)
    first = None
    shapes = [(w, s) for s in (bsg.BSG_SCHED_STRIDED, bsg.BSG_SCHED_RANGES) for w in (1, 3, 16, 64)]
    for w, s in shapes:
        nb = host(plan.compress(waves_per_cu=w, schedule=s)).copy()
        got = [host(o)[: m].copy() for o, m in zip(plan.outs, nb)]
        if first is None:
            first = (nb, got)
        else:
            assert np.array_equal(nb, first[0]), (w, s)
            assert all(np.array_equal(a, b) for a, b in zip(got, first[1])), (w, s)
    ns = [d.size // e for d, e in zip(data, Es)]
    dplan = bsg.BatchPlan.for_decompress(plan.outs, first[0].tolist(), ns, Es, Bs)
    for w, s in shapes:
        for o in dplan.outs:
            o.fill_(0xA5)
        assert not host(dplan.decompress(waves_per_cu=w, schedule=s)).any(), (w, s)
        for k, d in enumerate(data):
            assert np.array_equal(host(dplan.outs[k])[: d.size], d), (w, s, k)


def test_batch_unaligned_chunks(bsg):
    """Chunk inputs and outputs at odd addresses take the byte paths."""
    E, B = 4, 2048
    data = [chunk_data(k, E, 2048 * 2 + 5 + k) for k in range(4)]
    base = torch.zeros(sum(d.size for d in data) + 64, dtype=torch.uint8, device="cuda:0")
    xs, o = [], 1
    for d in data:
        base[o:o + d.size] = to_dev(d)
        xs.append(base[o:o + d.size])
        o += d.size + 3
    plan = bsg.BatchPlan.for_compress(xs, E, B)
    nb = host(plan.compress())
    for k, d in enumerate(data):
        ref = oracle.compress(d, E, B)
        assert nb[k] == ref.size and np.array_equal(host(plan.outs[k])[: ref.size], ref)
    big = torch.zeros(sum(d.size for d in data) + 64, dtype=torch.uint8, device="cuda:0")
    outs, o = [], 3
    for d in data:
        outs.append(big[o:o + d.size])
        o += d.size + 1
    dplan = bsg.BatchPlan.for_decompress(plan.outs, nb.tolist(), [d.size // E for d in data],
                                         E, B, outs=outs)
    assert not host(dplan.decompress()).any()
    for k, d in enumerate(data):
        assert np.array_equal(host(outs[k]), d)


def test_batch_capacity_is_per_chunk(bsg):
    data = [chunk_data(0, 4, 2048 * 4), chunk_data(2, 4, 2048 * 3), chunk_data(4, 4, 100)]
    refs = [oracle.compress(d, 4, 2048) for d in data]
    outs = [torch.empty(refs[0].size, dtype=torch.uint8, device="cuda:0"),
            torch.empty(refs[1].size - 1, dtype=torch.uint8, device="cuda:0"),
            torch.empty(16, dtype=torch.uint8, device="cuda:0")]  # below the fixed part
    plan = bsg.BatchPlan.for_compress([to_dev(d) for d in data], 4, 2048, outs=outs)
    nb = host(plan.compress())
    assert nb.tolist() == [refs[0].size, -2, -2]
    assert np.array_equal(host(outs[0]), refs[0])


def test_batch_corruption_is_per_chunk(bsg):
    E, B = 4, 2048
    x = synth.gen_gauss_int32(2048 * 8 + 5, 6, 2)
    s = oracle.compress(x, E, B)
    rng = np.random.default_rng(8)
    streams, lens, verdict = [], [], []
    for trial in range(24):
        c = s.copy()
        m = c.size
        kind = trial % 4
        if kind == 0:
            c[int(rng.integers(24 + 72, c.size))] ^= np.uint8(1 << int(rng.integers(0, 8)))
        elif kind == 1:
            c[int(rng.integers(24, 24 + 72))] ^= np.uint8(1 << int(rng.integers(0, 8)))
        elif kind == 2:
            m = int(rng.integers(24 + 72 + 28, c.size))
        # kind 3: intact
        try:
            ref = oracle.decompress(c[:m], x.size, E, B)
        except oracle.OracleError:
            ref = None
        streams.append(dev(c))
        lens.append(m)
        verdict.append(ref)
    dplan = bsg.BatchPlan.for_decompress(streams, lens, [x.size] * len(streams), E, B)
    st = host(dplan.decompress())
    for k, ref in enumerate(verdict):
        if ref is None:
            assert st[k] == -3, k
        else:
            assert st[k] == 0, k
            assert np.array_equal(host(dplan.outs[k]), ref.view(np.uint8).reshape(-1)), k
    assert sum(r is None for r in verdict) >= 8


def test_batch_graph_replay(bsg):
    """The batch calls enqueue only kernels: captured once, the graph replays
    to the oracle's bytes after the inputs change between replays."""
    data, Es, Bs = mixed()
    xs = [to_dev(d) for d in data]
    plan = bsg.BatchPlan.for_compress(xs, Es, Bs)
    nb0 = host(plan.compress())
    ns = [d.size // E for d, E in zip(data, Es)]
    dplan = bsg.BatchPlan.for_decompress(plan.outs, [int(v) for v in nb0], ns, Es, Bs)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.compress()
    for rep in range(3):
        new = [chunk_data(17 * rep + k, E, n) for k, (E, n) in enumerate(zip(Es, ns))]
        for x, d in zip(xs, new):
            if d.size:
                x.copy_(dev(d))
        torch.cuda.synchronize()
        g.replay()
        nb = host(plan.nbytes)
        for k, d in enumerate(new):
            ref = oracle.compress(d, Es[k], Bs[k])
            assert nb[k] == ref.size, (rep, k)
            assert np.array_equal(host(plan.outs[k])[: ref.size], ref), (rep, k)
        # eager decompression of the replayed streams (lengths changed)
        dp = bsg.BatchPlan.for_decompress(plan.outs, nb.tolist(), ns, Es, Bs)
        assert not host(dp.decompress()).any()
        for k, d in enumerate(new):
            assert np.array_equal(host(dp.outs[k])[: d.size], d), (rep, k)


def test_batch_decompress_graph_replay(bsg):
    data, Es, Bs = mixed()
    refs = [oracle.compress(d, E, B) for d, E, B in zip(data, Es, Bs)]
    ns = [d.size // E for d, E in zip(data, Es)]
    dplan = bsg.BatchPlan.for_decompress([dev(r) for r in refs], [r.size for r in refs], ns, Es, Bs)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        dplan.decompress()
    for rep in range(3):
        for o in dplan.outs:
            o.fill_(0xA5 ^ rep)
        dplan.status.fill_(7)  # the graph clears the status itself
        torch.cuda.synchronize()
        g.replay()
        assert not host(dplan.status).any(), rep
        for k, d in enumerate(data):
            assert np.array_equal(host(dplan.outs[k])[: d.size], d), (rep, k)


def test_batch_side_streams_graph_replay(bsg):
    """A batch of more than 16384 blocks in several element classes splits
    its classes over the library's own streams (each class scanned,
    finished and packed while the next one encodes).  Captured in a graph,
    it replays to the eager bytes three times, with other work and
    synchronisations between the replays."""
    specs = [(4, 2048, 2048 * 9000 + 5), (2, 4096, 4096 * 8000 + 8), (1, 8192, 8192 * 10 + 3)]
    data = [chunk_data(k, E, n) for k, (E, _, n) in enumerate(specs)]
    Es = [E for E, _, _ in specs]
    Bs = [b for _, b, _ in specs]
    xs = [to_dev(d) for d in data]
    plan = bsg.BatchPlan.for_compress(xs, Es, Bs)
    nb0 = host(plan.compress()).copy()
    eager = [host(o)[: int(m)].copy() for o, m in zip(plan.outs, nb0)]
    for k in (1, 2):  # the smaller chunks against the oracle as well
        assert np.array_equal(eager[k], oracle.compress(data[k], Es[k], Bs[k])), k
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.compress()
    for rep in range(3):
        for o in plan.outs:
            o.fill_(rep)
        plan.nbytes.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(plan.nbytes), nb0), rep
        for k, o in enumerate(plan.outs):
            assert np.array_equal(host(o)[: int(nb0[k])], eager[k]), (rep, k)
        _ = (xs[0][:4096].float() * 2).sum().item()  # other work between replays
