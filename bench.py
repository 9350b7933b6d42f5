"""Benchmarks of the DSSS iteration on one MI355X.

Default (the headline): PageRank on an R-MAT graph of scale 25, edge factor 48
(a/b/c/d = 0.57/0.19/0.19/0.05, seeded, self-loops kept, duplicates removed),
FP32 values. One step = one synchronous PageRank iteration over the whole graph:
every edge word is streamed once, its source value gathered, reduced by
destination in LDS and the vertex update applied. The layout is autotuned, the
K timed iterations are one replay of a captured hipGraph. Prints one JSON line.

Other workloads (--mode): bfs, wcc (scale 22, ef 16, 32 intervals), ppr (64
seeds, scale 22), multi (256 graphs, scales 10..18), adjoint (scale 20, fwd to
1e-8 residual + backward), degree (scale 22 over 2^23 sparse ids, with and
without degreeing), hoststream (the headline graph with its edge stream in
host memory); --mode all runs every one (one JSON line each). The default run
also times batched PPR, forward+backward, the 256-graph launch, BFS and WCC
and reports them under "forms" on the headline's line (--no-forms: headline
only).

  python bench.py [--steps K] [--warmup W]
                  [--mode pagerank|bfs|wcc|ppr|multi|adjoint|degree|hoststream|all]
"""
import argparse
import hashlib
import json
import tempfile
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pagerank_rmat_s25_ef48.traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1510_06916_amd", "csrc", "iterate.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha():
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(cfg):
    """HBM bytes per iteration (FETCH_SIZE + WRITE_SIZE of the iteration's three
    kernels, scaled by the copy probe's reading) from committed rocprofv3 counter
    runs, if one was taken on the current kernel source with the same layout
    (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            entries = json.load(f).get("entries", [])
    except (OSError, ValueError, AttributeError):
        return None
    sha = kernel_sha()
    for t in entries:
        if t.get("kernel_sha") == sha and all(
                t["config"].get(k, False if k == "pairs" else None) == cfg.get(k, False if k == "pairs" else None)
                for k in ("interval", "tile", "chunk", "piece_chunks", "order", "relabel", "pairs")):
            return t.get("bytes_per_iter")
    return None


def cpu_baseline_pagerank(src_d, dst_d, n, stride):
    """Times the CPU oracle (single thread, FP64) for one PageRank iteration over
    every stride-th edge of the same graph (n unchanged)."""
    import oracle
    src = src_d[::stride].cpu().numpy()
    dst = dst_d[::stride].cpu().numpy()
    oracle.outdeg(1, src[:1] * 0)  # load the library outside the timed region
    t0 = time.perf_counter()
    oracle.pagerank(n, src, dst, iters=1)
    dt = time.perf_counter() - t0
    m = len(src)
    return {"value": m / dt / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": "one FP64 PageRank iteration of the single-threaded C oracle over %s "
                      "(%d edges, n=%d): %.1f s" % ("every edge" if stride == 1 else
                                                    "every %d-th edge" % stride, m, n, dt),
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def rmat(scale, ef, seed, dev):
    import rmatgen
    t0 = time.perf_counter()
    src, dst = rmatgen.rmat_edges_gpu(scale, ef, seed, device=dev)
    log("R-MAT scale %d ef %d seed %d: m=%d (%.1fs)" % (scale, ef, seed, src.numel(),
                                                       time.perf_counter() - t0))
    return src, dst


# ---------------------------------------------------------------------------
def bench_pagerank(args, dev):
    import torch
    from paper_1510_06916_amd import DSSS, copy_probe, read_probe, tune
    n = 1 << args.scale
    src, dst = rmat(args.scale, args.ef, args.seed, dev)
    if args.interval or args.tile or args.chunk:
        best = {"interval": args.interval, "tile": args.tile, "chunk": args.chunk,
                "piece_chunks": args.piece, "order": ("dst", "src").index(args.order),
                "relabel": int(args.relabel), "pairs": int(args.pairs), "candidates": 0}
    else:
        t0 = time.perf_counter()
        os.environ.setdefault("NXG_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "nxg_tune_cache.txt"))
        os.makedirs(os.path.dirname(os.environ["NXG_TUNE_CACHE"]), exist_ok=True)
        best = tune(src, dst, n)
        log("tuned in %.1fs: %s" % (time.perf_counter() - t0, json.dumps(best)))
    t0 = time.perf_counter()
    order = ("dst", "src")[best["order"]]
    pairs = bool(best.get("pairs", 0))
    g = DSSS.build(src, dst, n, interval=best["interval"], tile=best["tile"],
                   chunk=best["chunk"], order=order, relabel=bool(best["relabel"]), pairs=pairs)
    torch.cuda.synchronize()
    inf = g.info()
    log("built DSSS in %.2fs: %s" % (time.perf_counter() - t0, json.dumps(inf)))
    m = inf["m"]
    piece = best["piece_chunks"]
    x, st = g.pagerank(max(args.warmup, 1), dtype=torch.float32, piece_chunks=piece)
    out = torch.empty(n, dtype=torch.float32, device=dev)
    g.pagerank(args.steps, dtype=torch.float32, capture=True, out=out, piece_chunks=piece)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    x, st = g.pagerank(args.steps, dtype=torch.float32, capture=True, out=out, piece_chunks=piece)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    kern_ms = ev0.elapsed_time(ev1) / args.steps
    log("timed %d steps (one graph replay): wall %.3f ms/step, events %.3f ms/step" %
        (args.steps, ms_step, kern_ms))
    b_iter = 4.0 * m + 12.0 * n
    achieved = b_iter / (kern_ms * 1e-3) / 1e9
    log("sum(x) = %.9f" % float(x.double().sum()))
    x = None
    # the paper's own order (destination-sorted sub-shards), same geometry: with
    # natural ids (the DSSS of Sec. II-A as is) and with out-degree numbering
    dsss_ms = {}
    if not args.no_ablation:
        del g, x
        torch.cuda.empty_cache()
        for relabel in (False, True):
            if order == "dst" and bool(best["relabel"]) == relabel:
                continue
            g2 = DSSS.build(src, dst, n, interval=best["interval"], tile=best["tile"], chunk=best["chunk"],
                            relabel=relabel)
            out2 = torch.empty(n, dtype=torch.float32, device=dev)
            g2.pagerank(args.steps, dtype=torch.float32, capture=True, out=out2, piece_chunks=piece)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g2.pagerank(args.steps, dtype=torch.float32, capture=True, out=out2, piece_chunks=piece)
            torch.cuda.synchronize()
            dsss_ms[relabel] = (time.perf_counter() - t0) * 1e3 / args.steps
            log("destination-sorted sub-shards, %s: %.3f ms/step" % (
                "out-degree numbering" if relabel else "natural ids", dsss_ms[relabel]))
            del g2, out2
            torch.cuda.empty_cache()
    # the paper's comparison scheme: the edge list sorted by source, pushed into
    # global sums with atomics (coarse-grained, Sec. IV-B1)
    scatter_ms = None
    if not args.no_ablation:
        g3 = DSSS.build(src, dst, n, scatter=True)
        out3 = torch.empty(n, dtype=torch.float32, device=dev)
        g3.pagerank(1, dtype=torch.float32, out=out3, scatter=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g3.pagerank(4, dtype=torch.float32, out=out3, scatter=True)
        torch.cuda.synchronize()
        scatter_ms = (time.perf_counter() - t0) * 1e3 / 4
        log("coarse-grained source-sorted scatter (I=%d): %.3f ms/step" % (g3.info()["interval"], scatter_ms))
        del g3, out3
        torch.cuda.empty_cache()
    copy_gbs = copy_probe(1 << 30, 10)
    read_gbs = read_probe(1 << 31, 10)
    log("copy probe: %.0f GB/s, read probe: %.0f GB/s" % (copy_gbs, read_gbs))
    traffic = measured_traffic({"interval": inf["interval"], "tile": inf["tile"], "chunk": inf["chunk"],
                                "piece_chunks": piece, "order": order,
                                "relabel": bool(best["relabel"]), "pairs": pairs})
    res = {
        "metric": "PageRank GTEPS per iteration (R-MAT scale %d, ef %d)" % (args.scale, args.ef),
        "value": m / (ms_step * 1e-3) / 1e9,
        "unit": "GTEPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic R-MAT (a/b/c/d=0.57/0.19/0.19/0.05, Philox seed %d, dedup)" % args.seed,
        "config": {"workload": "pagerank-iteration rmat-s%d-ef%d" % (args.scale, args.ef),
                   "n": n, "m": m, "interval": inf["interval"], "P": inf["P"],
                   "tile": inf["tile"], "chunk": inf["chunk"], "piece_chunks": piece,
                   "order": order, "relabel": bool(best["relabel"]), "pairs": pairs,
                   "words": inf["n_words"], "damping": 0.85,
                   "tuned_candidates": best["candidates"],
                   "dst_sorted_natural_ids_ms_per_step": dsss_ms.get(False),
                   "dst_sorted_relabeled_ms_per_step": dsss_ms.get(True),
                   "coarse_scatter_ms_per_step": scatter_ms},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_iter": b_iter, "kernel_ms": kern_ms,
                     "copy_probe_gbs": copy_gbs, "read_probe_gbs": read_gbs},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_pagerank(src, dst, n, args.cpu_stride)
    return res


# ---------------------------------------------------------------------------
def bench_bfs_wcc(args, dev, which):
    import numpy as np
    import torch
    import rmatgen
    from paper_1510_06916_amd import DSSS
    scale, ef, seed, P = 22, 16, 2, 32
    n = 1 << scale
    src, dst = rmat(scale, ef, seed, dev)
    interval = n // P
    if which == "bfs":
        g = DSSS.build(src, dst, n, interval=interval, value_bytes=4, order=args.order,
                       relabel=bool(args.relabel))
        deg = torch.bincount(src.long(), minlength=n).cpu().numpy()
        roots = rmatgen.distinct_vertices(seed + 100, 16, n, eligible=deg > 0)
        g.bfs(int(roots[0]))  # warm-up
        rates, times, passes = [], [], []
        n_chunks = g.info()["n_chunks"]
        for r in roots.tolist():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lev, st = g.bfs(r)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            times.append(dt)
            rates.append(st["reached_edges"] / dt)
            passes.append(st["streamed_chunks"] / n_chunks)
        hm = len(rates) / sum(1.0 / r for r in rates)
        # the 16 searches at once (one 64-bit root set per vertex, 8-byte accumulators)
        del g
        torch.cuda.empty_cache()
        gm = DSSS.build(src, dst, n, interval=interval, value_bytes=8, order=args.order,
                        relabel=bool(args.relabel))
        gm.bfs_multi(roots.tolist())  # warm-up (makes the workspace)
        mtimes = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, mst = gm.bfs_multi(roots.tolist())
            torch.cuda.synchronize()
            mtimes.append(time.perf_counter() - t0)
        mt = float(np.median(mtimes))
        res = {"metric": "BFS TEPS (harmonic mean over 16 roots)", "value": hm / 1e9,
               "unit": "GTEPS", "n_gpus": 1, "dtype": "i32", "higher_is_better": True,
               "config": {"workload": "bfs rmat-s22-ef16 P=32", "n": n, "m": gm.m,
                          "mean_ms": 1e3 * float(np.mean(times)), "roots": len(roots),
                          "stream_passes_per_bfs": float(np.mean(passes)),
                          "all_roots_at_once_ms": mt * 1e3,
                          "all_roots_at_once_gteps": mst["reached_edges"] / mt / 1e9,
                          "all_roots_at_once_vs_one_by_one": float(np.sum(times)) / mt}}
    elif which == "scc":
        g = DSSS.build(src, dst, n, interval=interval, value_bytes=4, transpose=True,
                       order=args.order, relabel=bool(args.relabel))
        g.scc()  # warm-up (makes the workspace)
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lab, st = g.scc()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        dt = float(np.median(times))
        _, sizes = np.unique(lab.cpu().numpy(), return_counts=True)
        res = {"metric": "SCC time (colouring rounds, labels = smallest id per component)",
               "value": dt * 1e3, "unit": "ms", "n_gpus": 1, "dtype": "i32", "higher_is_better": False,
               "config": {"workload": "scc rmat-s22-ef16 P=32", "n": n, "m": g.m, "timing": "median of 3",
                          "rounds": st["iterations"], "changing_passes": st["changed_rounds"],
                          "stream_passes": st["streamed_chunks"] / g.info()["n_chunks"],
                          "components": int(len(sizes)), "largest_component": int(sizes.max())}}
    else:
        g = DSSS.build(src, dst, n, interval=interval, value_bytes=4, symmetrize=True,
                       order=args.order, relabel=bool(args.relabel))
        g.wcc()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lab, st = g.wcc()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res = {"metric": "WCC label propagation (edges x rounds per second)",
               "value": g.m * st["changed_rounds"] / dt / 1e9, "unit": "GTEPS", "n_gpus": 1,
               "dtype": "i32", "higher_is_better": True,
               "config": {"workload": "wcc rmat-s22-ef16 symmetrised P=32", "n": n,
                          "m_sym": g.m, "rounds": st["changed_rounds"], "ms": dt * 1e3,
                          "stream_passes": st["streamed_chunks"] / g.info()["n_chunks"]}}
    return res


def bench_ppr(args, dev):
    import torch
    import rmatgen
    from paper_1510_06916_amd import DSSS, tune
    scale, ef, seed, B, iters = 22, 16, 4, 64, 30
    n = 1 << scale
    src, dst = rmat(scale, ef, seed, dev)
    seeds = torch.from_numpy(rmatgen.distinct_vertices(seed + 100, B, n))
    # vector width (columns per pass), tile, interval, order and numbering from the tuner
    t0 = time.perf_counter()
    best = tune(src, dst, n, batch=B)
    log("batched tune in %.1fs: %s" % (time.perf_counter() - t0, json.dumps(best)))
    W = best["width"]
    gb = DSSS.build(src, dst, n, tile=best["tile"], interval=best["interval"], chunk=best["chunk"],
                    order=("dst", "src")[best["order"]], relabel=bool(best["relabel"]),
                    value_bytes=8 * W)

    # one captured graph per pass (its seed slice and output stay put)
    parts = [seeds[i:i + W].to(dev, dtype=torch.int32).contiguous() for i in range(0, B, W)]
    outs = [torch.empty((n, p.numel()), dtype=torch.float32, device=dev) for p in parts]

    def run_all(k):
        for p, o in zip(parts, outs):
            gb.ppr(p, k, out=o, capture=True)

    gb.ppr(parts[0], 2)  # warm-up
    run_all(iters)       # records the graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_all(iters)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    gp = DSSS.build(src, dst, n, order=args.order, relabel=bool(args.relabel))
    tele = torch.zeros(n, dtype=torch.float32, device=dev)
    out = torch.empty(n, dtype=torch.float32, device=dev)
    tele[int(seeds[0])] = 1.0
    gp.pagerank(iters, teleport=tele, out=out, capture=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(B):
        tele.zero_()
        tele[int(seeds[b])] = 1.0
        gp.pagerank(iters, teleport=tele, out=out, capture=True)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    # the last plain run had seed B - 1: its column of the batched result against it
    xb = outs[-1][:, -1].double()
    acc = float((xb - out.double()).abs().sum() / out.double().abs().sum())
    res = {"metric": "batched PPR edge-vector updates per second", "value": B * gb.m * iters / tb / 1e9,
           "unit": "G updates/s", "n_gpus": 1, "dtype": "f32", "higher_is_better": True,
           "config": {"workload": "ppr rmat-s22-ef16 B=64 30 iterations", "n": n, "m": gb.m,
                      "width": W, "tile": best["tile"], "interval": best["interval"],
                      "order": ("dst", "src")[best["order"]], "relabel": best["relabel"],
                      "tuned_candidates": best["candidates"],
                      "plain_order": args.order, "plain_relabel": int(args.relabel),
                      "batched_ms": tb * 1e3, "plain_64_runs_ms": tp * 1e3,
                      "speedup_vs_plain": tp / tb, "rel_l1_vs_plain_last_column": acc}}
    return res


def bench_multi(args, dev):
    import numpy as np
    import torch
    import rmatgen
    from paper_1510_06916_amd import DSSS, MultiDSSS
    rng = np.random.default_rng(4000)
    graphs = []
    for g in range(256):
        scale = int(rng.integers(10, 19))
        ef = int(rng.integers(8, 33))
        s, d = rmatgen.rmat_edges_gpu(scale, ef, 4000 + g, device=dev)
        graphs.append((s, d, 1 << scale))
    m_total = sum(int(s.numel()) for s, _, _ in graphs)
    mg = MultiDSSS.build(graphs, order=args.order, relabel=bool(args.relabel))
    # like the plain runs below: outputs allocated once, one untimed run of the
    # same 30 iterations (plans, workspaces and the recorded graph), then the
    # timed replay
    mouts = [torch.empty(n, dtype=torch.float32, device=dev) for _, _, n in graphs]
    mg.pagerank(30, out=mouts, capture=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, st = mg.pagerank(30, out=mouts, capture=True)
    torch.cuda.synchronize()
    tm = time.perf_counter() - t0
    plain = [DSSS.build(s, d, n, order=args.order, relabel=bool(args.relabel)) for s, d, n in graphs]
    outs = [torch.empty(n, dtype=torch.float32, device=dev) for _, _, n in graphs]
    for g, o in zip(plain, outs):
        g.pagerank(30, out=o, capture=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g, o in zip(plain, outs):
        g.pagerank(30, out=o, capture=True)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    acc = max(float((a.double() - b.double()).abs().sum() / b.double().abs().sum()) for a, b in zip(xs, outs))
    res = {"metric": "256-graph PageRank (30 iterations) edges per second", "value": m_total * 30 / tm / 1e9,
           "unit": "GTEPS", "n_gpus": 1, "dtype": "f32", "higher_is_better": True,
           "config": {"workload": "multi 256 rmat graphs s10..18 ef8..32", "m_total": m_total,
                      "order": args.order, "relabel": int(args.relabel),
                      "one_launch_per_iteration_ms": tm * 1e3, "device_ms": st["device_ms"],
                      "captured": True,
                      "plain_captured_runs_ms": tp * 1e3,
                      "speedup_vs_plain": tp / tm, "max_rel_l1_vs_plain": acc}}
    return res


def bench_degree(args, dev):
    """Degreeing: the scale-22 ef16 R-MAT graph scattered over 2^23 ids (half of
    them in no edge), built and iterated with and without NXG_BUILD_DEGREE."""
    import numpy as np
    import torch
    from paper_1510_06916_amd import DSSS
    scale, ef, seed = 22, 16, 6
    n = 1 << (scale + 1)
    src, dst = rmat(scale, ef, seed, dev)
    spread = torch.from_numpy(np.random.default_rng(seed + 100).permutation(n)[: 1 << scale]
                              .astype(np.int32)).to(dev)
    src, dst = spread[src.long()], spread[dst.long()]
    res = {"metric": "PageRank FP32 ms per iteration, sparse ids, with and without degreeing",
           "unit": "ms", "n_gpus": 1, "dtype": "f32", "higher_is_better": False,
           "config": {"workload": "degree rmat-s22-ef16 over 2^23 ids", "n_ids": n, "m": int(src.numel()),
                      "order": args.order, "relabel": int(args.relabel)}}
    for deg in (False, True):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = DSSS.build(src, dst, n, order=args.order, relabel=bool(args.relabel), degree=deg)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        out = torch.empty(n, dtype=torch.float32, device=dev)
        g.pagerank(20, capture=True, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.pagerank(20, capture=True, out=out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / 20
        key = "degreed" if deg else "plain"
        res["config"][key + "_build_s"] = tb
        res["config"][key + "_ms_per_iter"] = ms
        res["config"][key + "_vertices"] = g.info()["n_kept"]
        del g
    res["value"] = res["config"]["degreed_ms_per_iter"]
    return res


def bench_hoststream(args, dev):
    """The headline graph with its edge stream in pinned host memory
    (NXG_BUILD_HOST_STREAM): FP32 PageRank iterations streaming 6.3 GB of
    sub-shards from the host each, against the host-to-device copy rate."""
    import torch
    from paper_1510_06916_amd import DSSS
    n = 1 << args.scale
    src, dst = rmat(args.scale, args.ef, args.seed, dev)
    g = DSSS.build(src, dst, n, interval=16384, tile=16384, chunk=1024, order="src", relabel=True,
                   host_stream=True)
    del src, dst
    torch.cuda.empty_cache()
    inf = g.info()
    out = torch.empty(n, dtype=torch.float32, device=dev)
    g.pagerank(1, out=out)
    torch.cuda.synchronize()
    iters = 3
    t0 = time.perf_counter()
    g.pagerank(iters, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / iters
    stream_bytes = 4.0 * inf["n_words"]
    # host-to-device rate of one 1 GiB pinned copy (best of 3)
    a = torch.empty(1 << 28, dtype=torch.float32, pin_memory=True)
    b = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    best = 1e9
    for _ in range(3):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        b.copy_(a, non_blocking=True)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t1)
    h2d = (1 << 30) / best / 1e9
    res = {"metric": "PageRank iteration with the edge stream in host memory", "value": ms, "unit": "ms",
           "n_gpus": 1, "dtype": "f32", "higher_is_better": False,
           "config": {"workload": "hoststream rmat-s%d-ef%d" % (args.scale, args.ef), "n": n, "m": inf["m"],
                      "stream_gb": stream_bytes / 1e9, "stream_gbs": stream_bytes / (ms * 1e-3) / 1e9,
                      "h2d_copy_gbs": h2d, "gteps": inf["m"] / (ms * 1e-3) / 1e9}}
    return res


def bench_mpu(args, dev):
    """Mixed-phase update (Sec. III-B3, Alg. 7) with host memory as the slower
    tier, on the headline graph with natural ids (edge order from --order):
    FP32 PageRank iterations at budgets that keep Q of P source intervals in
    device memory, from Q = P (the SPU) to Q = 0 (the DPU). Beside each, the
    host bytes the schedule moved and the paper's I/O bound for the same Q
    (B_e = 4, B_a = 4, B_v = 4; its hubs hold (id, value) pairs per edge, these
    hold one dense FP64 array per tile and sub-shard)."""
    import torch
    from paper_1510_06916_amd import DSSS
    n = 1 << args.scale
    src, dst = rmat(args.scale, args.ef, args.seed, dev)
    I, T = 1 << (args.scale - 4), 16384
    g = DSSS.build(src, dst, n, interval=I, tile=T, chunk=1024, order=args.order)
    del src, dst
    torch.cuda.empty_cache()
    inf = g.info()
    m, P = inf["m"], inf["P"]
    out = torch.empty(n, dtype=torch.float32, device=dev)
    iters = 3
    rows = []
    for Q in (P, 3 * P // 4, P // 2, P // 4, 0):
        budget = Q * I * (2 * 4 + 8) + I * 4
        g.pagerank(1, out=out, mpu_budget=budget)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = g.pagerank(iters, out=out, mpu_budget=budget)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / iters
        rd, wr = st["host_read_bytes"] / iters, st["host_write_bytes"] / iters
        f = (P - Q) / P
        paper_rd = m * (4 + f * f * 8) + f * n * 4
        paper_wr = f * f * m * 8 + f * n * 4
        rows.append({"Q": st["resident_intervals"], "ms_per_iter": ms, "host_read_gb": rd / 1e9,
                     "host_write_gb": wr / 1e9, "host_gbs": (rd + wr) / (ms * 1e-3) / 1e9,
                     "paper_model_read_gb": paper_rd / 1e9, "paper_model_write_gb": paper_wr / 1e9})
        log("MPU Q=%d: %.2f ms/iter, host read %.2f GB write %.2f GB" % (rows[-1]["Q"], ms, rd / 1e9, wr / 1e9))
    # the same layout through the plain (all-resident) path
    g.pagerank(1, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.pagerank(iters, out=out)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) * 1e3 / iters
    mid = [r for r in rows if r["Q"] == P // 2][0]
    res = {"metric": "PageRank iteration with Q of P intervals resident (MPU)", "value": mid["ms_per_iter"],
           "unit": "ms", "n_gpus": 1, "dtype": "f32", "higher_is_better": False,
           "config": {"workload": "mpu rmat-s%d-ef%d natural ids" % (args.scale, args.ef), "n": n,
                      "order": args.order,
                      "m": m, "P": P, "interval": I, "tile": T, "value_at_Q": P // 2, "iterations": iters,
                      "plain_path_ms_per_iter": plain_ms,
                      "by_Q": rows}}
    return res


def bench_adjoint(args, dev):
    import numpy as np
    import torch
    import rmatgen
    from paper_1510_06916_amd import DSSS, WeightedPageRank, tune
    scale, ef, seed = 20, 16, 5
    n = 1 << scale
    src, dst = rmat(scale, ef, seed, dev)
    w = rmatgen.row_normalized_weights(src.cpu().numpy(), n, seed=seed + 100)
    gvec = torch.from_numpy(rmatgen.normal_f32(seed + 200, n).astype(np.float64)).to(dev)
    # the layout the tuner picks for the weighted FP64 forward; the transposed
    # graph of the backward takes the same geometry
    t0 = time.perf_counter()
    best = tune(src, dst, n, dtype=torch.float64, weights=torch.from_numpy(w))
    log("weighted tune in %.1fs: %s" % (time.perf_counter() - t0, json.dumps(best)))
    g = DSSS.build(src, dst, n, weights=torch.from_numpy(w), transpose=True, keep_perm=True,
                   interval=best["interval"], tile=best["tile"], chunk=best["chunk"],
                   order=("dst", "src")[best["order"]], relabel=bool(best["relabel"]))
    wt = torch.from_numpy(w).to(dev)

    def fwd():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = g.pagerank(100000, dtype=torch.float64, tol=1e-8, weighted=True)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, st

    def fwd_bwd():
        wt.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs = WeightedPageRank.apply(wt, None, g, 0.85, 1e-8)
        (xs * gvec).sum().backward()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    wt.requires_grad_(True)
    fwd()
    fwd_bwd()  # warm-up: plans, workspaces, first launches
    runs = [fwd() for _ in range(3)]
    tf = sorted(r[0] for r in runs)[1]
    st = runs[0][1]
    tfb = sorted(fwd_bwd() for _ in range(3))[1]
    res = {"metric": "weighted PageRank forward (1e-8) + adjoint backward time",
           "value": tfb * 1e3, "unit": "ms", "n_gpus": 1, "dtype": "f64", "higher_is_better": False,
           "config": {"workload": "adjoint rmat-s20-ef16 weighted", "n": n, "m": g.m,
                      "order": ("dst", "src")[best["order"]], "relabel": best["relabel"],
                      "tile": best["tile"], "interval": best["interval"], "chunk": best["chunk"],
                      "tuned_candidates": best["candidates"], "timing": "median of 3",
                      "forward_iterations": st["iterations"], "forward_alone_ms": tf * 1e3,
                      "fwd_bwd_over_fwd": tfb / tf}}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", default="pagerank",
                    choices=["pagerank", "bfs", "wcc", "scc", "ppr", "multi", "adjoint", "degree",
                             "hoststream", "mpu", "all"])
    ap.add_argument("--scale", type=int, default=25)
    ap.add_argument("--ef", type=int, default=48)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--interval", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--piece", type=int, default=0, help="chunks per work item (0: automatic)")
    ap.add_argument("--order", default="src", choices=["dst", "src"])
    ap.add_argument("--relabel", type=int, default=1, help="with explicit layout flags: 1 = relabel")
    ap.add_argument("--pairs", type=int, default=0, help="with explicit layout flags: 1 = pair layout")
    ap.add_argument("--cpu-stride", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip timing the destination-sorted layouts and the coarse scatter beside the tuned one")
    ap.add_argument("--no-forms", action="store_true",
                    help="headline only: skip the batched PPR, forward+backward, 256-graph, BFS, WCC and "
                         "SCC figures the default run adds to its line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the DSSS iteration runs on a single MI355X "
              "(nothing multi-GPU is built)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    dev = torch.device("cuda:0")
    modes = (["pagerank", "bfs", "wcc", "scc", "ppr", "multi", "adjoint", "degree", "hoststream", "mpu"]
             if args.mode == "all" else [args.mode])
    runners = {"pagerank": bench_pagerank, "bfs": lambda a, d: bench_bfs_wcc(a, d, "bfs"),
               "wcc": lambda a, d: bench_bfs_wcc(a, d, "wcc"), "scc": lambda a, d: bench_bfs_wcc(a, d, "scc"),
               "ppr": bench_ppr, "multi": bench_multi,
               "degree": bench_degree, "hoststream": bench_hoststream, "adjoint": bench_adjoint,
               "mpu": bench_mpu}
    for mode in modes:
        log("== mode %s" % mode)
        res = runners[mode](args, dev)
        torch.cuda.empty_cache()
        if mode == "pagerank" and args.mode == "pagerank" and not args.no_forms:
            # the rest of the metric on the same line: batched PPR and
            # forward+backward against the plain path, the many-graph launch, and
            # the BFS / WCC rates and the SCC time of the scale-22 graph
            res["forms"] = {}
            for name in ("ppr", "adjoint", "multi", "bfs", "wcc", "scc"):
                log("== form %s" % name)
                t0 = time.perf_counter()
                r = runners[name](args, dev)
                torch.cuda.empty_cache()
                res["forms"][name] = {"metric": r["metric"], "value": r["value"], "unit": r["unit"],
                                      "dtype": r["dtype"], **r["config"],
                                      "bench_s": round(time.perf_counter() - t0, 1)}
        print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
