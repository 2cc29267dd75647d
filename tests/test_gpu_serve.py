"""GPU tests of the serving loop: the payload pool matches the oracle,
every request's result is the same served alone (the plain per-request
path) and in the mix (continuous batching over several streams), under a
budget that makes requests wait for memory, and the request loop makes no
device allocation (everything comes from buffers built with the server)."""
import numpy as np
import pytest

import oracle
from paper_1503_00638_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N, F_FRAC = synth.N_SAMPLES_DEFAULT, 0.01


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1503_00638_amd as m
    from paper_1503_00638_amd import serve, workloads
    m.load()
    sizes = synth.gen_pool_sizes(12, seed=11, lo=1 << 18, hi=1 << 24)
    pool = workloads.make_pool(sizes, seed=500, device="cuda:0")
    return m, serve, workloads, sizes, pool


def test_pool_matches_oracle(env):
    m, serve, workloads, sizes, pool = env
    for e, size in list(zip(pool, sizes))[:6]:
        vis, autos = workloads.pool_raw_vis(size, e.seed, "cuda:0")
        v, a = vis.cpu().numpy(), autos.cpu().numpy()
        r = oracle.round_to_noise(v, a, N, F_FRAC).view(np.uint8).reshape(-1)[:size]
        assert np.array_equal(e.data.cpu().numpy(), r)
        ref = oracle.compress(r.copy(), 4, workloads.POOL_BLOCK_ELEMS)
        assert e.stream_len == ref.size and np.array_equal(e.stream.cpu().numpy(), ref)


def check_results(reqs, pool, kept):
    for r in reqs:
        e = pool[r.payload]
        out, x = kept[r.rid]
        if r.op == "compress":
            mlen = int(x.item())
            assert mlen == e.stream_len, r
            assert torch.equal(out[:mlen], e.stream), r
        else:
            assert int(x.item()) == 0, r
            assert torch.equal(out[: e.nbytes], e.data), r


@pytest.mark.parametrize("budget_mib", [4096, 80])
def test_same_alone_and_in_the_mix(env, budget_mib):
    m, serve, workloads, sizes, pool = env
    reqs = synth.gen_requests(4000.0, 0.08, sizes, seed=21)
    assert len(reqs) > 150
    srv = serve.Server(pool, "cuda:0", hbm_budget=budget_mib << 20, n_streams=4, max_batch=32)
    keep = [r.rid for r in reqs]
    res_b, kept_b, nb_b = srv.run(reqs, "batch", keep)
    res_s, kept_s, nb_s = srv.run(reqs, "single", keep)
    assert nb_s == len(reqs)
    assert nb_b < len(reqs)  # requests were served together
    check_results(reqs, pool, kept_b)
    check_results(reqs, pool, kept_s)
    for s in res_b + res_s:
        assert s.t_done >= s.t_admit >= s.t_arrival - 1e-3
    summ = serve.summarize(res_b, nb_b)
    assert summ["latency_ms"]["p99"] >= summ["latency_ms"]["p50"] > 0


def test_request_loop_allocates_nothing(env):
    m, serve, workloads, sizes, pool = env
    reqs = synth.gen_requests(4000.0, 0.05, sizes, seed=23)
    srv = serve.Server(pool, "cuda:0", hbm_budget=256 << 20, n_streams=4, max_batch=16)
    srv.run(reqs[:10], "batch")
    srv.run(reqs[:10], "single")
    torch.cuda.synchronize()
    before = torch.cuda.memory_stats()["allocation.all.allocated"]
    _, _, nb_b = srv.run(reqs, "batch")
    _, _, nb_s = srv.run(reqs, "single")
    torch.cuda.synchronize()
    assert torch.cuda.memory_stats()["allocation.all.allocated"] == before
    assert nb_s == len(reqs) and nb_b < len(reqs)


def test_request_over_budget_is_refused(env):
    m, serve, workloads, sizes, pool = env
    reqs = synth.gen_requests(1000.0, 0.02, sizes, seed=22)
    srv = serve.Server(pool, "cuda:0", hbm_budget=1 << 16)
    with pytest.raises(ValueError):
        srv.run(reqs, "batch")
