"""PageRank iteration throughput on an R-MAT scale-25, edge-factor-48 graph.

One step = one synchronous PageRank iteration (FP32 values and accumulation)
over the whole graph stored as destination-sorted sub-shards: every edge word
is streamed once, its source value gathered, reduced by destination in LDS and
the vertex update applied. Prints one JSON line (rank 0).

  python bench.py [--steps K] [--warmup W] [--scale 25] [--ef 48]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(src_d, dst_d, n, sample_stride, iters=1):
    """Times the CPU oracle (single thread, FP64) for one PageRank iteration over
    every sample_stride-th edge of the same graph (n unchanged)."""
    import numpy as np
    import oracle
    src = src_d[::sample_stride].cpu().numpy()
    dst = dst_d[::sample_stride].cpu().numpy()
    oracle.outdeg(n, src[:1])  # load the library outside the timed region
    t0 = time.perf_counter()
    oracle.pagerank(n, src, dst, iters=iters)
    dt = time.perf_counter() - t0
    m = len(src)
    return {"value": m * iters / dt / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": "1 FP64 PageRank iteration of the single-threaded C oracle over every "
                      "%d-th edge (%d edges, n=%d), %.1f s" % (sample_stride, m, n, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--scale", type=int, default=25)
    ap.add_argument("--ef", type=int, default=48)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--interval", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--order", default="dst", choices=["dst", "src"])
    ap.add_argument("--cpu-stride", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check", action="store_true", help="also check sampled vertices vs FP64")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the DSSS iteration runs on a single MI355X "
              "(multi-GPU sharding is described in DESIGN.md, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    import rmatgen
    from paper_1510_06916_amd import DSSS

    dev = torch.device("cuda:0")
    n = 1 << args.scale
    t0 = time.perf_counter()
    src, dst = rmatgen.rmat_edges_gpu(args.scale, args.ef, args.seed, device=dev)
    torch.cuda.synchronize()
    log("generated R-MAT scale %d ef %d: m=%d in %.1fs" % (args.scale, args.ef, src.numel(),
                                                           time.perf_counter() - t0))
    t0 = time.perf_counter()
    g = DSSS.build(src, dst, n, interval=args.interval, tile=args.tile, chunk=args.chunk,
                   order=args.order)
    torch.cuda.synchronize()
    inf = g.info()
    log("built DSSS in %.2fs: %s" % (time.perf_counter() - t0, json.dumps(inf)))
    m = inf["m"]

    x, st = g.pagerank(args.warmup, dtype=torch.float32)
    torch.cuda.synchronize()
    log("warmup done: %s" % json.dumps(st))
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    x, st = g.pagerank(args.steps, dtype=torch.float32)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    kern_ms = ev0.elapsed_time(ev1) / args.steps
    log("timed %d steps: wall %.3f ms/step, events %.3f ms/step, lib %.3f ms total" %
        (args.steps, ms_step, kern_ms, st["device_ms"]))
    b_iter = 4.0 * m + 12.0 * n
    achieved = b_iter / (kern_ms * 1e-3) / 1e9
    mass = float(x.double().sum())
    log("sum(x) = %.9f" % mass)
    out = {
        "metric": "PageRank GTEPS per iteration (R-MAT scale %d, ef %d)" % (args.scale, args.ef),
        "value": m / (ms_step * 1e-3) / 1e9,
        "unit": "GTEPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic R-MAT (a/b/c/d=0.57/0.19/0.19/0.05, Philox seed %d, dedup)" % args.seed,
        "config": {"workload": "pagerank-iteration rmat-s%d-ef%d" % (args.scale, args.ef),
                   "n": n, "m": m, "interval": inf["interval"], "P": inf["P"],
                   "tile": inf["tile"], "chunk": inf["chunk"], "damping": 0.85,
                   "order": args.order},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_iter": b_iter, "kernel_ms": kern_ms},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(src, dst, n, args.cpu_stride)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
