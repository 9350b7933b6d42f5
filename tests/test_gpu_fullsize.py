"""Parity at the full benchmark sizes, in the launch configurations bench.py
times: R-MAT scale 25 / ef 48 PageRank (tuned layout), scale 22 BFS and WCC,
64-seed batched PPR, 256 graphs in one launch per iteration, and the scale-20
weighted-PageRank adjoint. The scale-25 run is also compared end to end with 20
FP64 oracle iterations (a few minutes of one host core)."""
import numpy as np
import pytest
import torch

import oracle
import rmatgen
from paper_1510_06916_amd import DSSS, MultiDSSS, WeightedPageRank, tune
from gpu_util import rel_l1, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfg3(gpu_device):
    say("cfg3: generating R-MAT scale 25 ef 48 seed 3")
    src_d, dst_d = rmatgen.rmat_edges_gpu(25, 48, 3, device=gpu_device)
    yield src_d, dst_d, src_d.cpu().numpy(), dst_d.cpu().numpy(), 1 << 25
    torch.cuda.empty_cache()


def test_cfg3_pagerank_fp32_tuned_layout(gpu_device, cfg3, progress):
    src_d, dst_d, src, dst, n = cfg3
    r = tune(src_d, dst_d, n)
    progress("cfg3 tuned layout: %s" % r)
    g = DSSS.build(src_d, dst_d, n, interval=r["interval"], tile=r["tile"], chunk=r["chunk"],
                   order=("dst", "src")[r["order"]], relabel=bool(r["relabel"]),
                   pairs=bool(r.get("pairs", 0)))
    pc = r["piece_chunks"]
    # one iteration from the uniform start, every vertex
    x1, _ = g.pagerank(1, dtype=torch.float32, piece_chunks=pc)
    progress("cfg3: oracle iteration 1")
    ref1, _ = oracle.pagerank(n, src, dst, iters=1)
    e1 = rel_l1(x1.cpu().numpy(), ref1)
    say("cfg3 iteration 1: rel L1 %.2e" % e1)
    assert e1 <= 1e-5
    # iteration 20 from the GPU's own iterate 19 (FP32 values upcast for the oracle)
    x19, _ = g.pagerank(19, dtype=torch.float32, piece_chunks=pc)
    x19h = x19.cpu().numpy().copy()
    x20, _ = g.pagerank(1, dtype=torch.float32, x0=x19, piece_chunks=pc)
    x20h = x20.cpu().numpy()
    progress("cfg3: oracle iteration 20 from the GPU iterate 19")
    ref20, _ = oracle.pagerank(n, src, dst, iters=1, x0=x19h.astype(np.float64))
    e20 = rel_l1(x20h, ref20)
    say("cfg3 iteration 20: rel L1 %.2e, mass %.9f" % (e20, float(x20h.astype(np.float64).sum())))
    assert e20 <= 1e-5
    assert abs(float(x20h.astype(np.float64).sum()) - 1.0) <= 1e-5
    # the captured 20-iteration run (what bench.py replays) gives the same vector
    out = torch.empty(n, dtype=torch.float32, device=gpu_device)
    xc, _ = g.pagerank(20, dtype=torch.float32, capture=True, out=out, piece_chunks=pc)
    assert rel_l1(xc.cpu().numpy(), x20h) <= 1e-6
    # end to end: the 20 FP32 iterations from the uniform start against 20 FP64
    # oracle iterations from the same start (about 10 s per oracle iteration; the
    # oracle continues from its own previous iterate, one iteration per call)
    ref20u = ref1
    for k in range(2, 21):
        ref20u, _ = oracle.pagerank(n, src, dst, iters=1, x0=ref20u)
        progress("cfg3: oracle iteration %d of 20 from the uniform start" % k)
    e20u = rel_l1(xc.cpu().numpy(), ref20u)
    progress("cfg3 20 iterations end to end: rel L1 %.2e" % e20u)
    assert e20u <= 1e-5


def test_cfg3_graph_bfs_level_properties(gpu_device, cfg3):
    # BFS on the 1.56G-edge graph (many activity segments): levels that hold at
    # any size -- the root at 0, no edge from a reached vertex skips a level, and
    # every other reached vertex has an in-edge from the level before it
    src_d, dst_d, _, _, n = cfg3
    g = DSSS.build(src_d, dst_d, n, value_bytes=4, order="src", relabel=True)
    s, d = src_d.long(), dst_d.long()
    root = int(torch.argmax(torch.bincount(s, minlength=n)))
    say("cfg3 bfs from %d" % root)
    lev, st = g.bfs(root)
    inf = 2**31 - 1
    lv = lev.long()
    ls, ld = lv[s], lv[d]
    fin = ls != inf
    assert int(lv[root]) == 0
    assert bool((ld[fin] <= ls[fin] + 1).all())
    has_parent = torch.zeros(n, dtype=torch.bool, device=gpu_device)
    has_parent[d[fin & (ld == ls + 1)]] = True
    reached = lv != inf
    reached[root] = False
    assert bool(has_parent[reached].all())
    assert st["max_level"] == int(lv[lv != inf].max()) and st["changed_rounds"] == st["max_level"]
    say("cfg3 bfs: %d levels, %d reached, %.2f stream passes" % (
        st["max_level"], int(reached.sum()) + 1, st["streamed_chunks"] / g.info()["n_chunks"]))


@pytest.fixture(scope="module")
def cfg2(gpu_device):
    src, dst = rmatgen.rmat_edges_gpu(22, 16, 2, device=gpu_device)
    n = 1 << 22
    src_h, dst_h = src.cpu().numpy(), dst.cpu().numpy()
    deg = np.bincount(src_h, minlength=n)
    roots = rmatgen.distinct_vertices(102, 16, n, eligible=deg > 0)
    # oracle results shared by the layouts below
    return {"src_d": src, "dst_d": dst, "src": src_h, "dst": dst_h, "n": n, "roots": roots,
            "bfs": {}, "wcc": None, "scc": None}


def _oracle_bfs(cfg, r):
    if r not in cfg["bfs"]:
        cfg["bfs"][r] = oracle.bfs(cfg["n"], cfg["src"], cfg["dst"], r)
    return cfg["bfs"][r]


# the layout bench.py times (source order, out-degree numbering, 32 intervals)
# with all 16 seeded roots, and the paper's DSSS order with natural ids
@pytest.mark.parametrize("order,relabel,nroots", [("src", True, 16), ("dst", False, 3)])
def test_cfg2_bfs_bit_exact(gpu_device, cfg2, order, relabel, nroots, progress):
    n = cfg2["n"]
    g = DSSS.build(cfg2["src_d"], cfg2["dst_d"], n, interval=n // 32, value_bytes=4, order=order,
                   relabel=relabel)
    for r in cfg2["roots"][:nroots].tolist():
        progress("cfg2 bfs order=%s relabel=%s root=%d" % (order, relabel, r))
        ref, rounds, mx = _oracle_bfs(cfg2, r)
        lev, st = g.bfs(r)
        assert np.array_equal(lev.cpu().numpy(), ref)
        assert st["changed_rounds"] == rounds and st["max_level"] == mx


def test_cfg2_bfs_all_roots_at_once(gpu_device, cfg2, progress):
    # the 16 searches in one run (one 64-bit root set per vertex), in the layout
    # the bench times them
    n = cfg2["n"]
    g = DSSS.build(cfg2["src_d"], cfg2["dst_d"], n, interval=n // 32, value_bytes=8, order="src",
                   relabel=True)
    roots = cfg2["roots"].tolist()
    progress("cfg2 bfs, 16 roots at once")
    lev, st = g.bfs_multi(roots)
    lev = lev.cpu().numpy()
    mx = 0
    for b, r in enumerate(roots):
        progress("cfg2 bfs column %d (root %d)" % (b, r))
        ref, rounds, m = _oracle_bfs(cfg2, r)
        assert np.array_equal(lev[:, b], ref)
        mx = max(mx, m)
    assert st["max_level"] == mx


@pytest.mark.parametrize("order,relabel", [("src", True), ("dst", False)])
def test_cfg2_wcc_bit_exact(gpu_device, cfg2, order, relabel, progress):
    n = cfg2["n"]
    g = DSSS.build(cfg2["src_d"], cfg2["dst_d"], n, interval=n // 32, value_bytes=4, symmetrize=True,
                   order=order, relabel=relabel)
    progress("cfg2 wcc order=%s relabel=%s" % (order, relabel))
    if cfg2["wcc"] is None:
        cfg2["wcc"] = oracle.wcc(n, cfg2["src"], cfg2["dst"])
    ref, rounds = cfg2["wcc"]
    lab, st = g.wcc()
    assert np.array_equal(lab.cpu().numpy(), ref)
    assert st["changed_rounds"] == rounds


@pytest.mark.parametrize("order,relabel", [("src", True), ("dst", False)])
def test_cfg2_scc_bit_exact(gpu_device, cfg2, order, relabel, progress):
    n = cfg2["n"]
    g = DSSS.build(cfg2["src_d"], cfg2["dst_d"], n, interval=n // 32, value_bytes=4, transpose=True,
                   order=order, relabel=relabel)
    progress("cfg2 scc order=%s relabel=%s" % (order, relabel))
    if cfg2["scc"] is None:
        cfg2["scc"] = oracle.scc(n, cfg2["src"], cfg2["dst"])
    ref, k = cfg2["scc"]
    lab, st = g.scc()
    lab = lab.cpu().numpy()
    assert np.array_equal(lab, ref)
    assert len(np.unique(lab)) == k and st["converged"] == 1


def test_cfg4_batched_ppr_64_seeds(gpu_device, progress):
    n = 1 << 22
    src_d, dst_d = rmatgen.rmat_edges_gpu(22, 16, 4, device=gpu_device)
    seeds = rmatgen.distinct_vertices(104, 64, n)
    gb = DSSS.build(src_d, dst_d, n, tile=256, interval=16384, value_bytes=8 * 64)
    say("cfg4 ppr: batched 64 x 30 iterations")
    xb, _ = gb.ppr(torch.from_numpy(seeds), 30)
    gp = DSSS.build(src_d, dst_d, n)
    tele = torch.zeros(n, dtype=torch.float32, device=gpu_device)
    worst = 0.0
    for b in range(64):
        tele.zero_()
        tele[int(seeds[b])] = 1.0
        xp, _ = gp.pagerank(30, teleport=tele)
        worst = max(worst, rel_l1(xb[:, b].cpu().numpy(), xp.cpu().numpy()))
    say("cfg4 ppr: worst column vs plain %.2e" % worst)
    assert worst <= 1e-6
    src_h, dst_h = src_d.cpu().numpy(), dst_d.cpu().numpy()
    for b in (0, 21, 42, 63):  # four columns against the FP64 oracle (about 10 s each)
        t = np.zeros(n)
        t[seeds[b]] = 1.0
        ref, _ = oracle.pagerank(n, src_h, dst_h, iters=30, t=t)
        e = rel_l1(xb[:, b].cpu().numpy(), ref)
        progress("cfg4 ppr: column %d vs oracle %.2e" % (b, e))
        assert e <= 1e-5


def test_cfg4_256_graphs(gpu_device):
    rng = np.random.default_rng(4000)
    graphs = []
    for gi in range(256):
        scale = int(rng.integers(10, 19))
        ef = int(rng.integers(8, 33))
        s, d = rmatgen.rmat_edges_gpu(scale, ef, 4000 + gi, device=gpu_device)
        graphs.append((s, d, 1 << scale))
    say("cfg4 multi: 256 graphs, %d edges" % sum(int(s.numel()) for s, _, _ in graphs))
    # the layout bench.py times: source order, out-degree numbering
    mg = MultiDSSS.build(graphs, order="src", relabel=True)
    xs, _ = mg.pagerank(30)
    worst = 0.0
    for gi, (s, d, n) in enumerate(graphs):
        xp, _ = DSSS.build(s, d, n).pagerank(30)
        worst = max(worst, rel_l1(xs[gi].cpu().numpy(), xp.cpu().numpy()))
    say("cfg4 multi: worst graph vs plain %.2e" % worst)
    assert worst <= 1e-6
    for gi in (0, 255):
        s, d, n = graphs[gi]
        ref, _ = oracle.pagerank(n, s.cpu().numpy(), d.cpu().numpy(), iters=30)
        assert rel_l1(xs[gi].cpu().numpy(), ref) <= 1e-5


def test_cfg5_adjoint_oracle_gradient_and_fd(gpu_device, progress):
    n = 1 << 20
    src_d, dst_d = rmatgen.rmat_edges_gpu(20, 16, 5, device=gpu_device)
    src, dst = src_d.cpu().numpy(), dst_d.cpu().numpy()
    w = rmatgen.row_normalized_weights(src, n, seed=105)
    gvec = rmatgen.normal_f32(205, n).astype(np.float64)
    g = DSSS.build(src_d, dst_d, n, weights=torch.from_numpy(w), transpose=True, keep_perm=True,
                   order="src", relabel=True)
    wt = torch.from_numpy(w).to(gpu_device).requires_grad_(True)
    tt = torch.full((n,), 1.0 / n, dtype=torch.float64, device=gpu_device, requires_grad=True)
    say("cfg5: forward to 1e-8 and backward")
    x = WeightedPageRank.apply(wt, tt, g, 0.85, 1e-8)
    (x * torch.from_numpy(gvec).to(gpu_device)).sum().backward()
    progress("cfg5: oracle forward to 1e-15")
    w64 = w.astype(np.float64)
    xs_ref, _ = oracle.pagerank(n, src, dst, iters=100000, w=w64, tol=1e-15)
    progress("cfg5: oracle adjoint")
    _, gw_ref, gt_ref, _ = oracle.pagerank_adjoint(n, src, dst, w64, xs_ref, gvec, tol=1e-12)
    ex = rel_l1(x.detach().cpu().numpy(), xs_ref)
    egw = rel_l1(wt.grad.cpu().numpy(), gw_ref)
    egt = rel_l1(tt.grad.cpu().numpy(), gt_ref)
    say("cfg5: x* %.2e  dL/dw %.2e  dL/dt %.2e" % (ex, egw, egt))
    # the forward stops at residual 1e-8: x* carries ~d/(1-d) * 1e-8 of error
    assert ex <= 1e-7
    assert egw <= 1e-6 and egt <= 1e-6
    # central differences on 1,000 sampled edges at h = 1e-4 (absolute). Each
    # perturbed forward is FP64, warm-started from x* and run a fixed 250
    # iterations (0.85^250 ~ 2e-18 of the start's distance is left), so the
    # truncation of a stopping test does not enter L; the O(h^2) term is
    # ~(h / w)^2 ~ 3e-6 relative at w ~ 1/16
    xstar = x.detach()
    gd = torch.from_numpy(gvec).to(gpu_device)
    picks = np.random.default_rng(5).choice(len(src), 1000, replace=False)
    h = 1e-4
    out = torch.empty(n, dtype=torch.float64, device=gpu_device)
    fd = []
    for i, e in enumerate(picks):
        le = []
        for sgn in (1.0, -1.0):
            wp = wt.detach().clone()
            wp[e] += sgn * h
            g.set_weights(wp)
            xp, _ = g.pagerank(250, dtype=torch.float64, weighted=True, x0=xstar, out=out, capture=True)
            le.append(float((xp * gd).sum()))
        he = float(np.float32(w[e] + h)) - float(np.float32(w[e] - h))
        fd.append((le[0] - le[1]) / he)
        if i % 100 == 99:
            progress("cfg5: central differences, %d of 1000 edges" % (i + 1))
    fd = np.array(fd)
    ad = wt.grad.cpu().numpy().astype(np.float64)[picks]
    err = np.linalg.norm(fd - ad) / np.linalg.norm(fd)
    worst = float(np.max(np.abs(fd - ad) / (np.abs(ad) + 1e-12)))
    say("cfg5: central differences on 1000 edges, rel L2 %.2e, worst per-edge %.2e" % (err, worst))
    assert err <= 1e-4
    # per edge, with an absolute floor far below the typical |dL/dw| ~ 1e-6
    assert np.all(np.abs(fd - ad) <= 1e-3 * np.abs(ad) + 1e-11)
