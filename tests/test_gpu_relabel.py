"""Builds with NXG_BUILD_RELABEL (vertices numbered internally by decreasing
out-degree): every program still takes and returns data in the caller's ids and
matches the oracle to the same bar as the plain build."""
import numpy as np
import pytest
import torch

import oracle
import rmatgen
from paper_1510_06916_amd import DSSS, MultiDSSS, WeightedPageRank
from gpu_util import rel_l1, say, to_dev

pytestmark = pytest.mark.gpu


def _graph(scale, ef, seed):
    src, dst = rmatgen.rmat_edges(scale, ef, seed=seed)
    return src, dst, 1 << scale


def test_vertex_map_and_structure(gpu_device):
    src, dst, n = _graph(12, 8, 21)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=512, tile=512,
                   relabel=True, keep_perm=True)
    assert g.info()["relabeled"] == 1
    n2o = g.vertex_map().cpu().numpy()
    assert np.array_equal(np.sort(n2o), np.arange(n))
    deg = np.bincount(src, minlength=n)
    # decreasing out-degree, ties by increasing caller id
    want = np.lexsort((np.arange(n), -deg))
    assert np.array_equal(n2o, want)
    o2n = np.empty(n, np.int64)
    o2n[n2o] = np.arange(n)
    s2, d2 = o2n[src].astype(np.int32), o2n[dst].astype(np.int32)
    perm_o, off_o = oracle.dsss_order(n, s2, d2, 512)
    ex = g.export(perm=True)
    assert np.array_equal(ex["offsets"].cpu().numpy(), off_o)
    assert np.array_equal(ex["perm"].cpu().numpy(), perm_o)
    assert np.array_equal(ex["src"].cpu().numpy(), s2[perm_o])
    assert np.array_equal(ex["dst"].cpu().numpy(), d2[perm_o])


@pytest.mark.parametrize("order", ["dst", "src"])
def test_pagerank_fp64_and_fp32(gpu_device, order):
    src, dst, n = _graph(16, 16, 1)
    ref, _ = oracle.pagerank(n, src, dst, iters=10)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, P=4, relabel=True,
                   order=order)
    say("relabel pagerank order=%s" % order)
    x, _ = g.pagerank(10, dtype=torch.float64)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12
    x32, _ = g.pagerank(10, dtype=torch.float32)
    assert rel_l1(x32.cpu().numpy(), ref) <= 1e-5
    out = torch.empty(n, dtype=torch.float32, device=gpu_device)
    for _ in range(3):  # captured graph replays, with eager work in between
        xc, _ = g.pagerank(10, dtype=torch.float32, capture=True, out=out)
        torch.cuda.synchronize()
        assert rel_l1(xc.cpu().numpy(), ref) <= 1e-5
        g.pagerank(2, dtype=torch.float32)


def test_teleport_tolerance_warm_start_weighted(gpu_device):
    src, dst, n = _graph(12, 8, 7)
    rng = np.random.default_rng(5)
    t = rng.random(n)
    t /= t.sum()
    w = rmatgen.row_normalized_weights(src, n, seed=33)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=1024,
                   weights=torch.from_numpy(w), keep_perm=True, relabel=True)
    say("relabel teleport/tol/warm start/weighted")
    ref, res = oracle.pagerank(n, src, dst, iters=200, t=t, tol=1e-10)
    x, st = g.pagerank(200, dtype=torch.float64, tol=1e-10, teleport=torch.from_numpy(t))
    assert st["converged"] == 1 and st["iterations"] == len(res)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12
    r12, _ = oracle.pagerank(n, src, dst, iters=12, t=t)
    x7, _ = g.pagerank(7, dtype=torch.float64, teleport=torch.from_numpy(t))
    x12, _ = g.pagerank(5, dtype=torch.float64, teleport=torch.from_numpy(t), x0=x7)
    assert rel_l1(x12.cpu().numpy(), r12) <= 1e-12
    rw, _ = oracle.pagerank(n, src, dst, iters=15, w=w.astype(np.float64))
    xw, _ = g.pagerank(15, dtype=torch.float64, weighted=True)
    assert rel_l1(xw.cpu().numpy(), rw) <= 1e-12


def test_bfs_and_wcc_bit_exact(gpu_device):
    src, dst, n = _graph(13, 8, 13)
    deg = np.bincount(src, minlength=n)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=1024,
                   relabel=True, value_bytes=4)
    roots = rmatgen.distinct_vertices(113, 3, n, eligible=deg > 0)
    for r in roots.tolist() + [int(np.flatnonzero(deg == 0)[0])]:
        say("relabel bfs root=%d" % r)
        ref, rounds, mx = oracle.bfs(n, src, dst, r)
        lev, st = g.bfs(r)
        assert np.array_equal(lev.cpu().numpy(), ref)
        assert st["changed_rounds"] == rounds and st["max_level"] == mx
        assert st["reached_edges"] == int(deg[ref != oracle.INF].sum())
    gs = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=1024,
                    relabel=True, symmetrize=True, value_bytes=4)
    say("relabel wcc")
    ref, rounds = oracle.wcc(n, src, dst)
    lab, st = gs.wcc()
    assert np.array_equal(lab.cpu().numpy(), ref)
    assert st["changed_rounds"] == rounds


def test_batched_ppr(gpu_device):
    src, dst, n = _graph(12, 8, 4)
    seeds = rmatgen.distinct_vertices(104, 16, n)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=1024, tile=256,
                   value_bytes=8 * 16, relabel=True)
    say("relabel ppr B=16")
    x, _ = g.ppr(torch.from_numpy(seeds), 12)
    x = x.cpu().numpy()
    for b in (0, 7, 15):
        t = np.zeros(n)
        t[seeds[b]] = 1.0
        ref, _ = oracle.pagerank(n, src, dst, iters=12, t=t)
        assert rel_l1(x[:, b], ref) <= 1e-5


def test_multi_graph(gpu_device):
    graphs, refs = [], []
    for k, (scale, ef) in enumerate([(10, 8), (12, 16), (11, 4)]):
        s, d = rmatgen.rmat_edges(scale, ef, seed=300 + k)
        graphs.append((to_dev(s, gpu_device), to_dev(d, gpu_device), 1 << scale))
        refs.append(oracle.pagerank(1 << scale, s, d, iters=9)[0])
    say("relabel multi 3 graphs")
    mg = MultiDSSS.build(graphs, relabel=True)
    xs, _ = mg.pagerank(9)
    for x, ref in zip(xs, refs):
        assert rel_l1(x.cpu().numpy(), ref) <= 1e-5


def test_adjoint(gpu_device):
    src, dst, n = _graph(11, 8, 5)
    w = rmatgen.row_normalized_weights(src, n, seed=105)
    gvec = rmatgen.normal_f32(205, n).astype(np.float64)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=512,
                   weights=torch.from_numpy(w), transpose=True, keep_perm=True, relabel=True)
    say("relabel adjoint")
    w64 = w.astype(np.float64)
    xs_ref, _ = oracle.pagerank(n, src, dst, iters=5000, w=w64, tol=1e-15)
    _, gw_ref, gt_ref, _ = oracle.pagerank_adjoint(n, src, dst, w64, xs_ref, gvec, tol=1e-14)
    wt = torch.from_numpy(w).to(gpu_device).requires_grad_(True)
    tt = torch.full((n,), 1.0 / n, dtype=torch.float64, device=gpu_device, requires_grad=True)
    x = WeightedPageRank.apply(wt, tt, g, 0.85, 1e-13)
    assert rel_l1(x.detach().cpu().numpy(), xs_ref) <= 1e-11
    (x * torch.from_numpy(gvec).to(gpu_device)).sum().backward()
    assert rel_l1(wt.grad.cpu().numpy(), gw_ref) <= 1e-6
    assert rel_l1(tt.grad.cpu().numpy(), gt_ref) <= 1e-10
