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


def cpu_baseline(vis, autos, w, n_freq):
    import oracle
    oracle.build(force=False)
    threads = oracle.max_threads()
    v = np.ascontiguousarray(vis[:n_freq])
    a = np.ascontiguousarray(autos[:n_freq])
    nb = w["block_bytes"] // 4
    t0 = time.perf_counter()
    r = oracle.round_to_noise(v, a, w["N"], w["f"], nthreads=threads)
    s = oracle.compress(r, 4, nb, nthreads=threads)
    t1 = time.perf_counter()
    d = oracle.decompress(s, r.size * 2, 4, nb, nthreads=threads)
    t2 = time.perf_counter()
    assert np.array_equal(d, r.view(np.uint8).reshape(-1))
    U = v.nbytes
    return {"value": U / (t2 - t0) / 1e9, "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_freq} of {vis.shape[0]} frequencies ({U / 1e9:.3f} GB): "
                      f"round+compress {U / (t1 - t0) / 1e9:.3f} GB/s, decompress "
                      f"{U / (t2 - t1) / 1e9:.3f} GB/s, ratio {s.size / U:.4f}"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-freqs", type=int, default=256,
                    help="frequencies of the workload the CPU oracle baseline times")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counter scale)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path shards by "
              "block ranges with no exchange, see DESIGN.md", file=sys.stderr)
        return 2

    import torch

    import paper_1503_00638_amd as bsg
    from paper_1503_00638_amd import synth

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

    def step(evs=None):
        if evs:
            evs[0].record(stream)
        bsg.round_compress(dvis, dautos, w["N"], w["f"], nb, out=out, workspace=ws, nbytes=nbytes)
        if evs:
            evs[1].record(stream)
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
    # algorithmic bytes (SURVEY-style accounting): rounding+compress
    # reads U + autos and writes rU + offsets; decompress reads rU + offsets, writes U
    n_blocks = -(-n // nb)
    table = 8 * (n_blocks + 1)
    bytes_comp = U + autos.nbytes + m
    bytes_dec = m + U
    dominant, dom_ms, dom_bytes = ("k_encode+scan+pack (round_compress)", comp, bytes_comp) \
        if comp >= dcm else ("k_decode (decompress)", dcm, bytes_dec)
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = traffic_for("k_decode" if dominant.startswith("k_decode") else "k_encode")
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


if __name__ == "__main__":
    sys.exit(main())
