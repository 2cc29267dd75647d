"""Benchmark of the compression hot path on one MI355X.

A step is one pass of the whole path over one chunk already resident in
HBM: noise-relative rounding fused with bitshuffle + LZ4 compression
(round_compress), then decompression with the fused inverse bit transpose.
Workload: a CHIME-Pathfinder-shaped chunk of complex64 visibilities,
(1024 freq, 8256 products from 128 inputs, 32 times) = 2.16 GB, f = 0.01,
N = 3.9e6, 8192-byte blocks of float32 elements (synthetic, seeded).

Prints one JSON line (rank 0).  The headline value is uncompressed bytes per
second of the full step (compress + decompress); per-call rates, the
compression ratio, step latency percentiles, the roofline of the dominant
kernel and the CPU oracle baseline come with it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
WORKLOAD = dict(F=1024, I=128, T=32, seed=1, f=0.01, N=3.9e6, block_bytes=8192)


def source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1503_00638_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str):
    """HBM bytes per launch from committed rocprofv3 --pmc counters, if they
    were taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_digest") != source_digest():
        return None
    return rec.get("hbm_bytes_per_launch")


def host_description():
    """CPU model and core counts of the machine the oracle baseline runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0))}


def cpu_baseline(vis, autos, w, n_freq):
    """The oracle on the host's cores over the first n_freq frequencies:
    round + compress, then decompress, with the OpenMP thread count the
    process allows (blocks spread over threads) and with one thread (the
    setting of the paper's single-core figures)."""
    import oracle
    oracle.build(force=False)
    threads = oracle.max_threads()
    v = np.ascontiguousarray(vis[:n_freq])
    a = np.ascontiguousarray(autos[:n_freq])
    nb = w["block_bytes"] // 4
    U = v.nbytes

    def run(nthreads):
        t0 = time.perf_counter()
        r = oracle.round_to_noise(v, a, w["N"], w["f"], nthreads=nthreads)
        s = oracle.compress(r, 4, nb, nthreads=nthreads)
        t1 = time.perf_counter()
        d = oracle.decompress(s, r.size * 2, 4, nb, nthreads=nthreads)
        t2 = time.perf_counter()
        assert np.array_equal(d, r.view(np.uint8).reshape(-1))
        return {"value": round(U / (t2 - t0) / 1e9, 4),
                "round_compress_GBps": round(U / (t1 - t0) / 1e9, 4),
                "decompress_GBps": round(U / (t2 - t1) / 1e9, 4), "ratio": round(s.size / U, 5)}

    multi = run(threads)
    single = run(1)
    return {"value": multi["value"], "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_freq} of {vis.shape[0]} frequencies ({U / 1e9:.3f} GB), "
                      f"round+compress then decompress: {threads} threads "
                      f"{multi['round_compress_GBps']:.3f} / {multi['decompress_GBps']:.3f} GB/s, "
                      f"1 thread {single['round_compress_GBps']:.3f} / "
                      f"{single['decompress_GBps']:.3f} GB/s, ratio {multi['ratio']:.4f}",
            "threads": multi, "single_thread": single, "host": host_description()}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-freqs", type=int, default=128,
                    help="frequencies of the workload the CPU oracle baseline times")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counter scale)")
    ap.add_argument("--workload", choices=("chunk", "batch", "serve", "sweep", "filters", "extensions"),
                    default="chunk",
                    help="chunk: one 2.16 GB CHIME-shaped chunk (default); batch: 4096 "
                         "independent chunks; serve: Poisson request stream; sweep: bit "
                         "transpose of 1 GiB at every element size and block size")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-sweep", type=float, nargs="*",
                    default=[2000.0, 5000.0, 10000.0, 20000.0, 40000.0, 80000.0],
                    help="request rates of the serving sweep (req/s)")
    ap.add_argument("--serve-sweep-requests", type=int, default=3000)
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): blocks, chunks and "
              "requests are independent, so the path would shard by block ranges or whole "
              "chunks with no exchange, but no multi-GPU run is part of this benchmark",
              file=sys.stderr)
        return 2

    import torch

    import paper_1503_00638_amd as bsg
    from paper_1503_00638_amd import synth

    if args.workload == "batch":
        return bench_batch(args, torch, bsg)
    if args.workload == "serve":
        return bench_serve(args, torch, bsg)
    if args.workload == "sweep":
        return bench_sweep(args, torch, bsg)
    if args.workload == "filters":
        return bench_filters(args, torch, bsg)
    if args.workload == "extensions":
        return bench_extensions(args, torch, bsg)

    w = WORKLOAD
    dev = torch.device("cuda:0")
    print(f"# generating workload F={w['F']} I={w['I']} T={w['T']}", file=sys.stderr, flush=True)
    vis, autos = synth.gen_vis(w["F"], w["I"], w["T"], w["seed"], w["N"])
    U = vis.nbytes
    n = 2 * vis.size
    nb = w["block_bytes"] // 4
    dvis = torch.from_numpy(vis).to(dev)
    dautos = torch.from_numpy(autos).to(dev)
    bound = bsg.compress_bound(n, 4, nb)
    out = torch.empty(bound, dtype=torch.uint8, device=dev)
    ws = torch.empty(bsg.workspace_size(n, 4, nb), dtype=torch.uint8, device=dev)
    nbytes = torch.empty(1, dtype=torch.int64, device=dev)
    dec = torch.empty(U, dtype=torch.uint8, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    rounded = torch.empty_like(dvis)
    stream = torch.cuda.current_stream()

    # first pass: stream length (deterministic) and correctness of the round trip
    bsg.round_compress(dvis, dautos, w["N"], w["f"], nb, out=out, workspace=ws, nbytes=nbytes)
    torch.cuda.synchronize()
    m = int(nbytes.item())
    assert m > 0
    bsg.decompress(out, m, n, 4, nb, out=dec, status=status)
    bsg.round_to_noise(dvis, dautos, w["N"], w["f"], out=rounded)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert torch.equal(dec, rounded.view(torch.uint8).reshape(-1)), "round trip mismatch"
    ratio = m / U

    def ev():
        return torch.cuda.Event(enable_timing=True)

    # roctx ranges (torch.cuda.nvtx maps to roctx on ROCm): a marker trace
    # (rocprofv3 --marker-trace) shows each step and its two calls
    rng = torch.cuda.nvtx.range

    def step(evs=None):
        with rng("step"):
            if evs:
                evs[0].record(stream)
            with rng("round_compress"):
                bsg.round_compress(dvis, dautos, w["N"], w["f"], nb, out=out, workspace=ws,
                                   nbytes=nbytes)
            if evs:
                evs[1].record(stream)
            with rng("decompress"):
                bsg.decompress(out, m, n, 4, nb, out=dec, status=status)
            if evs:
                evs[2].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[ev(), ev(), ev()] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    comp_ms = np.array([e[0].elapsed_time(e[1]) for e in evs])
    dec_ms = np.array([e[1].elapsed_time(e[2]) for e in evs])
    step_ms = comp_ms + dec_ms
    assert int(nbytes.item()) == m and int(status.item()) == 0

    # the standalone calls, for the per-stage report
    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    t_round = timed(lambda: bsg.round_to_noise(dvis, dautos, w["N"], w["f"], out=rounded))
    rflat = rounded.view(torch.uint8).reshape(-1)
    t_comp_plain = timed(lambda: bsg.compress(rflat, 4, nb, out=out, workspace=ws, nbytes=nbytes))
    t_shuf = timed(lambda: bsg.bitshuffle(rflat, 4, nb, out=dec))

    comp = float(np.mean(comp_ms))
    dcm = float(np.mean(dec_ms))
    # algorithmic bytes: rounding+compress reads U + autos and writes rU
    # (offsets included); decompress reads rU and writes U
    n_blocks = -(-n // nb)
    table = 8 * (n_blocks + 1)
    bytes_comp = U + autos.nbytes + m
    bytes_dec = m + U
    if comp >= dcm:
        dominant, dom_ms, dom_bytes, tkey = (
            "round_compress call: k_encode<8192,4,1> in 16 segments on two streams, "
            "k_tile_sum + k_tile_offsets + k_write_offsets + k_pack per segment on a third",
            comp, bytes_comp, "round_compress_call")
    else:
        dominant, dom_ms, dom_bytes, tkey = ("decompress call: k_decode<8192,4>", dcm, bytes_dec,
                                             "decompress_call")
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = traffic_for(tkey)
    value = U * args.steps / (float(np.sum(step_ms)) * 1e-3) / 1e9

    res = {
        "metric": "uncompressed GB/s (compress & decompress) + % HBM peak; p50/p99 latency",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(float(np.mean(step_ms)), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "CHIME-Pathfinder-shaped chunk: complex64 (1024 freq, 8256 products "
                               "from 128 inputs, 32 times), 2.16 GB, f=0.01, N=3.9e6, "
                               "round_to_noise+bitshuffle+LZ4 compress, then decompress",
                   "global_batch": 1, "block_bytes": w["block_bytes"], "elem_size": 4,
                   "parallelism": "single GPU"},
        "compress_GBps": round(U / (comp * 1e-3) / 1e9, 2),
        "decompress_GBps": round(U / (dcm * 1e-3) / 1e9, 2),
        "round_only_GBps": round(U / (t_round * 1e-3) / 1e9, 2),
        "compress_unfused_GBps": round(U / (t_comp_plain * 1e-3) / 1e9, 2),
        "bitshuffle_only_GBps": round(U / (t_shuf * 1e-3) / 1e9, 2),
        "ratio": round(ratio, 5),
        "hbm_frac_step": round((bytes_comp + bytes_dec) / (float(np.mean(step_ms)) * 1e-3) / 1e9
                               / HBM_PEAK_GBPS, 4),
        "hbm_frac_decompress": round(bytes_dec / (dcm * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "hbm_frac_compress": round(bytes_comp / (comp * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 4),
                       "p99": round(float(np.percentile(step_ms, 99)), 4),
                       "compress_p50": round(float(np.percentile(comp_ms, 50)), 4),
                       "decompress_p50": round(float(np.percentile(dec_ms, 50)), 4)},
        "wall_s_timed": round(wall, 4),
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_launch": int(dom_bytes)},
        "source_digest": source_digest(),
    }
    if args.calibrate_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu:
        print("# timing the CPU oracle baseline", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(vis, autos, w, min(args.cpu_freqs, w["F"]))
    print(json.dumps(res), flush=True)
    return 0


def _events(torch, n):
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def _time_calls(torch, fn, steps, warmup):
    """Per-call device times (ms) of fn on the current stream."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = _events(torch, steps + 1)
    ev[0].record(stream)
    for k in range(steps):
        fn()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    return np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])


def bench_batch(args, torch, bsg):
    """Many independent chunks: the batch entry points (one persistent
    kernel per element class, captured in a graph, launch shape autotuned)
    against the plain per-chunk calls on the same buffers."""
    from paper_1503_00638_amd import tune, workloads

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    specs, xs = workloads.make_batch(args.batch_count, device=dev)
    torch.cuda.synchronize()
    print(f"# generated {len(specs)} chunks in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    Es = [s.elem_size for s in specs]
    Bs = [8192 // e for e in Es]
    ns = [s.nbytes // s.elem_size for s in specs]
    U = sum(s.nbytes for s in specs)

    plan_c = bsg.BatchPlan.for_compress(xs, Es, Bs)
    wc, tune_c = tune.tune(plan_c, "compress", use_cache=False)
    nb = plan_c.compress(*wc).cpu().numpy().copy()
    assert (nb > 0).all()
    plan_d = bsg.BatchPlan.for_decompress(plan_c.outs, nb.tolist(), ns, Es, Bs)
    wd, tune_d = tune.tune(plan_d, "decompress", use_cache=False)
    st = plan_d.decompress(*wd)
    torch.cuda.synchronize()
    assert not st.any().item()
    for x, y, s in zip(xs, plan_d.outs, specs):
        assert torch.equal(x, y[: s.nbytes]), f"round trip mismatch in chunk {s.index}"
    print(f"# tuned (waves/CU, schedule): compress {wc}, decompress {wd}", file=sys.stderr,
          flush=True)

    gc, gd = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(gc):
        plan_c.compress(*wc)
    with torch.cuda.graph(gd):
        plan_d.decompress(*wd)
    comp_ms = _time_calls(torch, gc.replay, args.steps, args.warmup)
    dec_ms = _time_calls(torch, gd.replay, args.steps, args.warmup)
    assert np.array_equal(plan_c.nbytes.cpu().numpy(), nb) and not plan_d.status.any().item()

    # the plain per-chunk path on the same data (own output buffers)
    outs = [torch.empty_like(o) for o in plan_c.outs]
    ws = torch.empty(max(bsg.workspace_size(n, e, b) for n, e, b in zip(ns, Es, Bs)),
                     dtype=torch.uint8, device=dev)
    nbytes_pc = torch.empty(len(xs), dtype=torch.int64, device=dev)
    status_pc = torch.zeros(len(xs), dtype=torch.int32, device=dev)
    dec_pc = [torch.empty_like(o) for o in plan_d.outs]

    def per_chunk_compress():
        for k, x in enumerate(xs):
            bsg.compress(x, Es[k], Bs[k], out=outs[k], workspace=ws, nbytes=nbytes_pc[k:k + 1])

    def per_chunk_decompress():
        for k in range(len(xs)):
            bsg.decompress(outs[k], int(nb[k]), ns[k], Es[k], Bs[k], out=dec_pc[k],
                           status=status_pc[k:k + 1])

    pc_steps = max(1, min(args.steps, 3))
    pcc_ms = _time_calls(torch, per_chunk_compress, pc_steps, 1)
    pcd_ms = _time_calls(torch, per_chunk_decompress, pc_steps, 1)
    assert np.array_equal(nbytes_pc.cpu().numpy(), nb), "per-chunk lengths differ from batch"
    for k in range(len(xs)):
        assert torch.equal(outs[k][: nb[k]], plan_c.outs[k][: nb[k]]), f"stream {k} differs"
    assert not status_pc.any().item()
    gpc_c, gpc_d = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.graph(gpc_c):
        per_chunk_compress()
    with torch.cuda.graph(gpc_d):
        per_chunk_decompress()
    gpcc_ms = _time_calls(torch, gpc_c.replay, pc_steps, 1)
    gpcd_ms = _time_calls(torch, gpc_d.replay, pc_steps, 1)

    C = float(nb.sum())
    comp, dcm = float(np.median(comp_ms)), float(np.median(dec_ms))
    gbps = lambda ms: round(U / (ms * 1e-3) / 1e9, 2)
    enc_bytes, dec_bytes = U + C, C + U
    dominant = ("k_batch_encode+scan+finish+pack (batch compress)", comp, enc_bytes) \
        if comp >= dcm else ("k_batch_decode+k_batch_dec_tail (batch decompress)", dcm, dec_bytes)
    achieved = dominant[2] / (dominant[1] * 1e-3) / 1e9
    res = {
        "metric": "uncompressed GB/s (compress & decompress) + % HBM peak; p50/p99 latency",
        "value": round(U / ((comp + dcm) * 1e-3) / 1e9, 2),
        "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(comp + dcm, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"batched: {len(xs)} independent chunks, sizes log-uniform "
                               f"64 KiB-64 MiB (total {U / 2**30:.2f} GiB), elem_size in {{2,4,8}}, "
                               "half noise-rounded visibilities, half int16 random walks, "
                               "8192-byte blocks; batch compress then batch decompress, "
                               "each one captured graph",
                   "chunks": len(xs), "total_bytes": U, "parallelism": "single GPU"},
        "compress_GBps": gbps(comp), "decompress_GBps": gbps(dcm),
        "ratio": round(C / U, 5),
        "hbm_frac_compress": round(enc_bytes / (comp * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "hbm_frac_decompress": round(dec_bytes / (dcm * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "latency_ms": {"compress_p50": round(float(np.percentile(comp_ms, 50)), 3),
                       "compress_p99": round(float(np.percentile(comp_ms, 99)), 3),
                       "decompress_p50": round(float(np.percentile(dec_ms, 50)), 3),
                       "decompress_p99": round(float(np.percentile(dec_ms, 99)), 3)},
        "autotune": {"knobs": "waves_per_cu,schedule (0 strided, 1 contiguous ranges)",
                     "best": {"compress": list(wc), "decompress": list(wd)},
                     "compress_ms": {str(k): round(v, 3) for k, v in tune_c.items()},
                     "decompress_ms": {str(k): round(v, 3) for k, v in tune_d.items()}},
        "per_chunk_eager": {"compress_GBps": gbps(float(np.median(pcc_ms))),
                            "decompress_GBps": gbps(float(np.median(pcd_ms)))},
        "per_chunk_graph": {"compress_GBps": gbps(float(np.median(gpcc_ms))),
                            "decompress_GBps": gbps(float(np.median(gpcd_ms)))},
        "roofline": {"bound": "hbm", "kernel": dominant[0], "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                     "algorithmic_bytes_per_launch": int(dominant[2])},
        "source_digest": source_digest(),
    }
    print(json.dumps(res), flush=True)
    return 0


def bench_sweep(args, torch, bsg):
    """Bit transpose only, 1 GiB per call: forward and inverse at element
    sizes 1/2/4/8/16 and block sizes of 2048/8192/65536 bytes.  Each call
    reads and writes 1 GiB (2 GiB of HBM traffic)."""
    dev = torch.device("cuda:0")
    nbytes = 1 << 30
    g = torch.Generator(device=dev).manual_seed(2)
    x = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device=dev, generator=g)
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    rows = []
    for E in (1, 2, 4, 8, 16):
        for bb in (2048, 8192, 65536):
            nb = bb // E
            fwd = _time_calls(torch, lambda: bsg.bitshuffle(x, E, nb, out=y), args.steps,
                              args.warmup)
            inv = _time_calls(torch, lambda: bsg.bitunshuffle(y, E, nb, out=z), args.steps,
                              args.warmup)
            torch.cuda.synchronize()
            assert torch.equal(x, z), (E, bb)
            f, i = float(np.median(fwd)), float(np.median(inv))
            rows.append({"elem_size": E, "block_bytes": bb,
                         "forward_GBps": round(nbytes / (f * 1e-3) / 1e9, 1),
                         "inverse_GBps": round(nbytes / (i * 1e-3) / 1e9, 1),
                         "forward_hbm_frac": round(2 * nbytes / (f * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                         "inverse_hbm_frac": round(2 * nbytes / (i * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)})
    # a plain device-to-device copy of the same size: the achievable ceiling
    cp = float(np.median(_time_calls(torch, lambda: z.copy_(x), args.steps, args.warmup)))
    copy_gbps = 2 * nbytes / (cp * 1e-3) / 1e9
    best = max(rows, key=lambda r: r["forward_GBps"])
    worst = min(rows, key=lambda r: min(r["forward_GBps"], r["inverse_GBps"]))
    res = {
        "metric": "uncompressed GB/s (compress & decompress) + % HBM peak; p50/p99 latency",
        "value": round(float(np.median([min(r["forward_GBps"], r["inverse_GBps"]) for r in rows])), 1),
        "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "bit-transpose sweep: 1 GiB of uniform random bytes per call, "
                               "elem_size 1/2/4/8/16 x block 2048/8192/65536 bytes, "
                               "bitshuffle and bitunshuffle (value: median over the 15 cases "
                               "of the slower direction)",
                   "parallelism": "single GPU"},
        "cases": rows,
        "copy_hbm_GBps": round(copy_gbps, 1),
        "roofline": {"bound": "hbm", "kernel": f"bitshuffle E={best['elem_size']} "
                                               f"B={best['block_bytes']}",
                     "achieved": round(2 * best["forward_GBps"], 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": best["forward_hbm_frac"], "traffic": None,
                     "algorithmic_bytes_per_launch": 2 * nbytes},
        "slowest_case": worst,
        "source_digest": source_digest(),
    }
    print(json.dumps(res), flush=True)
    return 0


def bench_filters(args, torch, bsg):
    """The paper's comparison (Table t:performance): the same rounded
    CHIME-shaped chunk compressed with the bit transpose and with the
    Blosc-style byte shuffle before the same LZ4; ratio and throughput."""
    from paper_1503_00638_amd import synth

    w = WORKLOAD
    dev = torch.device("cuda:0")
    vis, autos = synth.gen_vis(w["F"], w["I"], w["T"], w["seed"], w["N"])
    dvis, dautos = torch.from_numpy(vis).to(dev), torch.from_numpy(autos).to(dev)
    r = bsg.round_to_noise(dvis, dautos, w["N"], w["f"]).view(torch.uint8).reshape(-1)
    del dvis
    U = r.numel()
    n, nb = U // 4, w["block_bytes"] // 4
    out = torch.empty(bsg.compress_bound(n, 4, nb), dtype=torch.uint8, device=dev)
    ws = torch.empty(bsg.workspace_size(n, 4, nb), dtype=torch.uint8, device=dev)
    nbytes = torch.empty(1, dtype=torch.int64, device=dev)
    dec = torch.empty(U, dtype=torch.uint8, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    rows = {}
    for name, flt in (("bitshuffle", bsg.BSG_FILTER_BIT), ("byteshuffle", bsg.BSG_FILTER_BYTE)):
        bsg.compress(r, 4, nb, out=out, workspace=ws, nbytes=nbytes, filter=flt)
        m = int(nbytes.item())
        c_ms = _time_calls(torch, lambda: bsg.compress(r, 4, nb, out=out, workspace=ws,
                                                         nbytes=nbytes, filter=flt),
                           args.steps, args.warmup)
        d_ms = _time_calls(torch, lambda: bsg.decompress(out, m, n, 4, nb, out=dec, status=status,
                                                           filter=flt), args.steps, args.warmup)
        torch.cuda.synchronize()
        assert int(status.item()) == 0 and torch.equal(dec, r), name
        # the filter alone (no LZ4), forward then inverse
        fwd, inv = ((bsg.bitshuffle, bsg.bitunshuffle) if flt == bsg.BSG_FILTER_BIT
                    else (bsg.byteshuffle, bsg.byteunshuffle))
        f_ms = _time_calls(torch, lambda: fwd(r, 4, nb, out=dec), args.steps, args.warmup)
        i_ms = _time_calls(torch, lambda: inv(dec, 4, nb, out=out[:U]), args.steps, args.warmup)
        torch.cuda.synchronize()
        assert torch.equal(out[:U], r), name
        rows[name] = {"ratio": round(m / U, 5),
                      "compress_GBps": round(U / (float(np.median(c_ms)) * 1e-3) / 1e9, 2),
                      "decompress_GBps": round(U / (float(np.median(d_ms)) * 1e-3) / 1e9, 2),
                      "filter_only_GBps": round(U / (float(np.median(f_ms)) * 1e-3) / 1e9, 2),
                      "inverse_only_GBps": round(U / (float(np.median(i_ms)) * 1e-3) / 1e9, 2)}
    res = {
        "metric": "uncompressed GB/s (compress & decompress) + % HBM peak; p50/p99 latency",
        "value": rows["bitshuffle"]["decompress_GBps"], "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "filter comparison: the rounded CHIME-Pathfinder-shaped chunk "
                               "(2.16 GB, f=0.01) with the bit transpose vs the Blosc-style byte "
                               "shuffle before the same per-block LZ4, 8192-byte blocks",
                   "parallelism": "single GPU"},
        "filters": rows,
        "paper_ratios_for_context": {"bitshuffle_lz4": 0.279, "blosc_lz4": 0.473},
        "source_digest": source_digest(),
    }
    print(json.dumps(res), flush=True)
    return 0


def bench_extensions(args, torch, bsg):
    """The rows beyond the float path, on the CHIME-Pathfinder shape (1024
    freq, 8256 products, 32 times): integer visibilities (int32 re/im, the
    correlator's own type) rounded and compressed as 8-byte elements, and
    the compensation of the diagonal noise model (factor, then rounding
    with it) on point-source-dominated visibilities."""
    from paper_1503_00638_amd import synth

    w = WORKLOAD
    dev = torch.device("cuda:0")
    F, I, T = w["F"], w["I"], w["T"]
    res_rows = {}
    # integer visibilities: the float model scaled by 1024 and rounded
    vis, autos = synth.gen_vis_device(F, I, T, w["seed"], w["N"], device=dev)
    vi = torch.round(torch.view_as_real(vis) * 1024.0).to(torch.int32)
    pairs = torch.from_numpy(synth.product_pairs(I)).to(dev)
    ai = vi[..., 0][:, pairs[:, 0] == pairs[:, 1], :].contiguous()
    del vis, autos
    U = vi.numel() * 4
    ro = torch.empty_like(vi)
    t_round = float(np.median(_time_calls(
        torch, lambda: bsg.round_to_noise_i32(vi, ai, w["N"], w["f"], out=ro), args.steps,
        args.warmup)))
    flat = ro.view(torch.uint8).reshape(-1)
    n8, nb8 = U // 8, w["block_bytes"] // 8
    out = torch.empty(bsg.compress_bound(n8, 8, nb8), dtype=torch.uint8, device=dev)
    ws = torch.empty(bsg.workspace_size(n8, 8, nb8), dtype=torch.uint8, device=dev)
    nbytes = torch.empty(1, dtype=torch.int64, device=dev)
    t_comp = float(np.median(_time_calls(
        torch, lambda: bsg.compress(flat, 8, nb8, out=out, workspace=ws, nbytes=nbytes), args.steps,
        args.warmup)))
    m = int(nbytes.item())
    dec = torch.empty(U, dtype=torch.uint8, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    t_dec = float(np.median(_time_calls(
        torch, lambda: bsg.decompress(out, m, n8, 8, nb8, out=dec, status=st), args.steps,
        args.warmup)))
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and torch.equal(dec, flat)
    res_rows["integer_visibilities"] = {
        "round_GBps": round(U / (t_round * 1e-3) / 1e9, 2),
        "round_hbm_frac": round((2 * U + ai.numel() * 4) / (t_round * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "compress_e8_GBps": round(U / (t_comp * 1e-3) / 1e9, 2),
        "decompress_e8_GBps": round(U / (t_dec * 1e-3) / 1e9, 2), "ratio": round(m / U, 5)}
    del vi, ai, ro, flat, out, ws, dec
    # compensation: a source adding 40 % of the receiver power to every product
    vis, autos = synth.gen_vis_device(F, I, T, w["seed"], w["N"], device=dev)
    vr = torch.view_as_real(vis)
    vr[..., 0] += 400.0
    autos += 400.0
    U = vis.numel() * 8
    scale = torch.empty((F, T), dtype=torch.float64, device=dev)
    t_fac = float(np.median(_time_calls(
        torch, lambda: bsg.noise_compensation(vis, autos, out=scale), args.steps, args.warmup)))
    rout = torch.empty_like(vis)
    t_rs = float(np.median(_time_calls(
        torch, lambda: bsg.round_to_noise_scaled(vis, autos, w["N"], w["f"], scale, out=rout),
        args.steps, args.warmup)))
    res_rows["noise_compensation"] = {
        "factor_GBps": round(U / (t_fac * 1e-3) / 1e9, 2),
        "factor_hbm_frac": round((U + autos.numel() * 4) / (t_fac * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "factor_min": round(float(scale.min().item()), 6),
        "scaled_round_GBps": round(U / (t_rs * 1e-3) / 1e9, 2)}
    del vis, autos, vr, rout, scale
    # full-covariance noise for small arrays: per sample a D x D covariance,
    # D = I^2, factorised and inverted in LDS (2 D^3 / 3 flops for the
    # Cholesky factor and the triangular inverse, D^2 for the diagonal)
    fc = {}
    for Ic, Fc, Tc in ((8, 1024, 64), (11, 256, 64)):
        vis, autos = synth.gen_vis_device(Fc, Ic, Tc, w["seed"], w["N"], device=dev)
        out_fc = torch.empty_like(vis)
        t_fc = float(np.median(_time_calls(
            torch, lambda: bsg.round_to_noise_fullcov(vis, autos, w["N"], w["f"], out=out_fc),
            args.steps, args.warmup)))
        D = Ic * Ic
        samples = Fc * Tc
        fc[f"I{Ic}"] = {"samples": samples, "dof_per_sample": D, "ms": round(t_fc, 3),
                        "samples_per_s": round(samples / (t_fc * 1e-3), 1),
                        "GBps": round(vis.numel() * 8 / (t_fc * 1e-3) / 1e9, 2),
                        "fp64_TFLOPs": round(samples * (2 * D ** 3 / 3) / (t_fc * 1e-3) / 1e12, 3)}
        del vis, autos, out_fc
    res_rows["full_covariance"] = fc
    res = {
        "metric": "uncompressed GB/s (compress & decompress) + % HBM peak; p50/p99 latency",
        "value": res_rows["integer_visibilities"]["round_GBps"], "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "i32/f64", "data": "synthetic",
        "config": {"workload": "integer visibilities and noise-model compensation on the "
                               "CHIME-Pathfinder shape (1024 freq, 8256 products, 32 times), "
                               "f=0.01, N=3.9e6, 8192-byte blocks; full-covariance rounding "
                               "for small arrays (8 inputs x 1024 freq x 64 times, 11 inputs x "
                               "256 freq x 64 times)",
                   "parallelism": "single GPU"},
        "rows": res_rows, "source_digest": source_digest(),
    }
    print(json.dumps(res), flush=True)
    return 0


def bench_serve(args, torch, bsg):
    """Poisson request stream over a device-resident payload pool: the
    continuous-batching loop against the plain per-request path, at the
    workload's rate (the headline) and over a sweep of rates up to
    saturation."""
    from paper_1503_00638_amd import serve, synth, workloads

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    sizes = synth.gen_pool_sizes(256, seed=4)
    pool = workloads.make_pool(sizes, device=dev)
    for e in pool:  # every payload's stream decodes back to it
        out, st = bsg.decompress(e.stream, e.stream_len, e.n, 4, workloads.POOL_BLOCK_ELEMS)
        assert torch.equal(out[: e.nbytes], e.data) and int(st.item()) == 0
    print(f"# pool of {len(pool)} payloads ({sum(sizes) / 2**30:.2f} GiB) in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    reqs = synth.gen_requests(args.serve_rate, args.serve_seconds, sizes, seed=5)
    budget = 64 << 30
    srv = serve.Server(pool, dev, hbm_budget=budget, n_streams=4, max_batch=64)
    warm = [r for r in reqs[:300]]
    srv.run(warm, "batch")
    srv.run(warm, "single")
    keep = {r.rid for r in reqs[::97]}
    res_b, kept_b, nb_b = srv.run(reqs, "batch", keep)
    print("# batched run done", file=sys.stderr, flush=True)
    res_s, kept_s, nb_s = srv.run(reqs, "single", keep)
    print("# per-request run done", file=sys.stderr, flush=True)
    by_id = {r.rid: r for r in reqs}
    for rid in keep:  # same bytes alone and in the mix, and equal to the pool
        r, e = by_id[rid], pool[by_id[rid].payload]
        (ob, xb), (os_, xs) = kept_b[rid], kept_s[rid]
        if r.op == "compress":
            m = int(xb.item())
            assert m == int(xs.item()) == e.stream_len
            assert torch.equal(ob[:m], os_[:m]) and torch.equal(ob[:m], e.stream)
        else:
            assert int(xb.item()) == 0 and int(xs.item()) == 0
            assert torch.equal(ob[: e.nbytes], e.data) and torch.equal(os_[: e.nbytes], e.data)
    sb, ss = serve.summarize(res_b, nb_b), serve.summarize(res_s, nb_s)
    sweep = []
    for rate in args.serve_sweep:
        n_req = int(args.serve_sweep_requests)
        rq = synth.gen_requests(rate, n_req / rate, sizes, seed=6)
        row = {"rate_per_s": rate, "offered_GBps": round(sum(r.nbytes for r in rq) / (n_req / rate)
                                                         / 1e9, 1)}
        for mode in ("batch", "single"):
            res, _, nb = srv.run(rq, mode)
            sm = serve.summarize(res, nb)
            row[mode] = {"p50_ms": sm["latency_ms"]["p50"], "p99_ms": sm["latency_ms"]["p99"],
                         "sustained_GBps": sm["sustained_GBps"], "launches": nb}
        sweep.append(row)
        print(f"# rate {rate}/s: batch {row['batch']}, single {row['single']}", file=sys.stderr,
              flush=True)
    res = {
        "metric": "uncompressed GB/s (compress & decompress) + % HBM peak; p50/p99 latency",
        "value": sb["sustained_GBps"], "unit": "GB/s", "n_gpus": 1,
        "steps": len(reqs), "warmup": len(warm), "ms_per_step": sb["latency_ms"]["mean"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"serving: Poisson arrivals at {args.serve_rate:g}/s for "
                               f"{args.serve_seconds:g} s, 60/40 decompress/compress, payloads of "
                               "noise-rounded CHIME-shaped visibilities (float32 elements, "
                               "8192-byte blocks), 256 KiB-256 MiB log-uniform, 64 GiB HBM "
                               "budget for outputs and workspaces in flight, continuous "
                               "batching on 4 streams",
                   "pool_payloads": len(pool), "hbm_budget": budget,
                   "parallelism": "single GPU"},
        "batched": sb, "per_request": ss,
        "rate_sweep": {"requests_per_rate": int(args.serve_sweep_requests), "rows": sweep},
        "source_digest": source_digest(),
    }
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
