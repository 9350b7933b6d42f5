"""Degreeing (NXG_BUILD_DEGREE): ids that appear in no edge are dropped and the
rest numbered densely. Every program must equal the oracle run on the compacted
graph, expanded back to the caller's ids (dropped ids: 0 for PageRank and the
adjoint, INT32_MAX for BFS, their own id for WCC)."""
import numpy as np
import pytest
import torch

import oracle
import rmatgen
from paper_1510_06916_amd import DSSS, NxgError, WeightedPageRank
from gpu_util import rel_l1, say, to_dev

pytestmark = pytest.mark.gpu

N = 10000


def _sparse_graph(seed):
    s, d = rmatgen.rmat_edges(12, 8, seed=seed)
    spread = np.random.default_rng(seed).permutation(N)[:4096]  # ids 0..4095 -> sparse ids
    return spread[s].astype(np.int32), spread[d].astype(np.int32)


def _compact(src, dst):
    used = np.zeros(N, bool)
    used[src] = True
    used[dst] = True
    kept = np.flatnonzero(used)
    o2n = np.full(N, -1, np.int64)
    o2n[kept] = np.arange(len(kept))
    return kept, o2n, o2n[src].astype(np.int32), o2n[dst].astype(np.int32)


@pytest.mark.parametrize("relabel", [False, True])
def test_pagerank_bfs_and_map(gpu_device, relabel):
    src, dst = _sparse_graph(61)
    kept, o2n, s2, d2 = _compact(src, dst)
    nk = len(kept)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), N, interval=1024, degree=True,
                   relabel=relabel, keep_perm=True)
    say("degree relabel=%s: n=%d kept=%d" % (relabel, N, nk))
    inf = g.info()
    assert inf["n"] == N and inf["n_kept"] == nk
    n2o = g.vertex_map().cpu().numpy()
    assert np.array_equal(np.sort(n2o), kept)
    if not relabel:
        assert np.array_equal(n2o, kept)
    ref_c, _ = oracle.pagerank(nk, s2, d2, iters=10)
    ref = np.zeros(N)
    ref[kept] = ref_c
    x, _ = g.pagerank(10, dtype=torch.float64)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12
    x32, _ = g.pagerank(10, dtype=torch.float32)
    assert rel_l1(x32.cpu().numpy(), ref) <= 1e-5
    # teleport counts only on kept ids
    t = np.random.default_rng(3).random(N)
    t /= t.sum()
    rt_c, _ = oracle.pagerank(nk, s2, d2, iters=6, t=t[kept])
    rt = np.zeros(N)
    rt[kept] = rt_c
    xt, _ = g.pagerank(6, dtype=torch.float64, teleport=torch.from_numpy(t))
    assert rel_l1(xt.cpu().numpy(), rt) <= 1e-12
    # BFS from a kept root and from a dropped one
    gb = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), N, interval=1024, degree=True,
                    relabel=relabel, value_bytes=4)
    root = int(src[0])
    lev_c, rounds, mx = oracle.bfs(nk, s2, d2, int(o2n[root]))
    want = np.full(N, oracle.INF, np.int64)
    want[kept] = lev_c
    lev, st = gb.bfs(root)
    assert np.array_equal(lev.cpu().numpy(), want)
    assert st["changed_rounds"] == rounds and st["max_level"] == mx
    dropped = int(np.flatnonzero(o2n < 0)[0])
    lev0, _ = gb.bfs(dropped)
    l0 = lev0.cpu().numpy()
    assert l0[dropped] == 0 and np.all(np.delete(l0, dropped) == oracle.INF)


def test_wcc_and_batched_ppr(gpu_device):
    src, dst = _sparse_graph(62)
    kept, o2n, s2, d2 = _compact(src, dst)
    nk = len(kept)
    gs = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), N, interval=1024, degree=True,
                    symmetrize=True, value_bytes=4)
    lab_c, rounds = oracle.wcc(nk, s2, d2)
    want = np.arange(N)
    want[kept] = kept[lab_c]  # the compacted order keeps caller order, so minima agree
    lab, st = gs.wcc()
    assert np.array_equal(lab.cpu().numpy(), want)
    assert st["changed_rounds"] == rounds
    gp = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), N, interval=1024, tile=512,
                    degree=True, value_bytes=8 * 8)
    seeds = kept[np.random.default_rng(9).choice(nk, 8, replace=False)]
    xb, _ = gp.ppr(torch.from_numpy(seeds.astype(np.int32)), 10)
    xb = xb.cpu().numpy()
    for b in (0, 5):
        t = np.zeros(nk)
        t[o2n[seeds[b]]] = 1.0
        r_c, _ = oracle.pagerank(nk, s2, d2, iters=10, t=t)
        r = np.zeros(N)
        r[kept] = r_c
        assert rel_l1(xb[:, b], r) <= 1e-5
    dropped = int(np.flatnonzero(o2n < 0)[0])
    with pytest.raises(NxgError, match="EINVAL"):
        gp.ppr(torch.tensor([int(seeds[0]), dropped], dtype=torch.int32), 3)


def test_adjoint(gpu_device):
    src, dst = _sparse_graph(63)
    kept, o2n, s2, d2 = _compact(src, dst)
    nk = len(kept)
    # weights normalised over each source's out-edges
    w = rmatgen.row_normalized_weights(src, N, seed=163)
    gvec = rmatgen.normal_f32(263, N).astype(np.float64)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), N, interval=1024, degree=True,
                   weights=torch.from_numpy(w), transpose=True, keep_perm=True)
    w64 = w.astype(np.float64)
    xs_c, _ = oracle.pagerank(nk, s2, d2, iters=5000, w=w64, tol=1e-15)
    _, gw_ref, gt_c, _ = oracle.pagerank_adjoint(nk, s2, d2, w64, xs_c, gvec[kept], tol=1e-14)
    wt = torch.from_numpy(w).to(gpu_device).requires_grad_(True)
    tt = torch.zeros(N, dtype=torch.float64, device=gpu_device)
    tt[torch.from_numpy(kept).to(gpu_device)] = 1.0 / nk
    tt.requires_grad_(True)
    x = WeightedPageRank.apply(wt, tt, g, 0.85, 1e-13)
    xs = np.zeros(N)
    xs[kept] = xs_c
    assert rel_l1(x.detach().cpu().numpy(), xs) <= 1e-11
    (x * torch.from_numpy(gvec).to(gpu_device)).sum().backward()
    gt_ref = np.zeros(N)
    gt_ref[kept] = gt_c
    assert rel_l1(wt.grad.cpu().numpy(), gw_ref) <= 1e-6
    assert rel_l1(tt.grad.cpu().numpy(), gt_ref) <= 1e-10


@pytest.mark.parametrize("relabel", [False, True])
def test_pagerank_pair_layout(gpu_device, relabel):
    # degreeing then the pair layout: PageRank over the compacted graph, in the
    # caller's ids
    src, dst = _sparse_graph(63)
    kept, o2n, s2, d2 = _compact(src, dst)
    nk = len(kept)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), N, interval=512, tile=1024,
                   chunk=256, degree=True, relabel=relabel, order="src", pairs=True)
    assert g.info()["pairs"] == 1 and g.info()["n_kept"] == nk
    ref_c, _ = oracle.pagerank(nk, s2, d2, iters=9)
    ref = np.zeros(N)
    ref[kept] = ref_c
    x, _ = g.pagerank(9, dtype=torch.float64)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12


def test_multi_refuses_degree(gpu_device):
    from paper_1510_06916_amd import _lib
    import ctypes
    d = (_lib.BuildDesc * 1)()
    d[0] = _lib.BuildDesc(n=10, m=0, flags=_lib.NXG_BUILD_DEGREE)
    h = ctypes.c_void_p()
    assert _lib.lib().nxg_multi_build(1, d, None, ctypes.byref(h)) == _lib.NXG_EUNSUPPORTED
