"""BFS levels and WCC labels on the GPU against the oracle, bit-exact."""
import numpy as np
import pytest

import oracle
import rmatgen
from paper_1510_06916_amd import DSSS
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("scale,interval,tile,order,relabel", [
    (12, 512, 0, "dst", False), (13, 8192, 1024, "dst", False), (14, 1000, 0, "dst", False),
    (14, 700, 8192, "dst", False), (13, 1024, 4096, "src", False), (14, 2048, 0, "src", True)])
def test_bfs_bit_exact(gpu_device, scale, interval, tile, order, relabel):
    n = 1 << scale
    src, dst = rmatgen.rmat_edges(scale, 8, seed=scale)
    deg = np.bincount(src, minlength=n)
    roots = rmatgen.distinct_vertices(scale + 100, 4, n, eligible=deg > 0)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=interval, tile=tile,
                   order=order, relabel=relabel)
    for r in roots.tolist() + [int(np.flatnonzero(deg == 0)[0])]:
        say("bfs scale=%d I=%d root=%d" % (scale, interval, r))
        ref, rounds, mx = oracle.bfs(n, src, dst, r)
        lev, st = g.bfs(r)
        assert np.array_equal(lev.cpu().numpy(), ref)
        assert st["changed_rounds"] == rounds and st["max_level"] == mx
        assert st["reached_edges"] == int(deg[ref != oracle.INF].sum())


@pytest.mark.parametrize("scale,interval,order,relabel", [
    (12, 512, "dst", False), (14, 2048, "dst", False), (13, 1024, "src", False), (14, 4096, "src", True)])
def test_wcc_bit_exact(gpu_device, scale, interval, order, relabel):
    n = 1 << scale
    src, dst = rmatgen.rmat_edges(scale, 4, seed=scale + 50)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=interval,
                   symmetrize=True, order=order, relabel=relabel)
    say("wcc scale=%d I=%d" % (scale, interval))
    ref, rounds = oracle.wcc(n, src, dst)
    lab, st = g.wcc()
    assert np.array_equal(lab.cpu().numpy(), ref)
    assert st["changed_rounds"] == rounds


def test_bfs_path_graph(gpu_device):
    n = 3000
    src = np.arange(n - 1, dtype=np.int32)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(src + 1, gpu_device), n, interval=128)
    lev, st = g.bfs(0)
    assert np.array_equal(lev.cpu().numpy(), np.arange(n))
    assert st["changed_rounds"] == n - 1 and st["max_level"] == n - 1


@pytest.mark.parametrize("n,tile,interval,order", [
    (1000, 16, 128, "dst"), (1000, 32, 256, "src"), (1777, 8, 64, "dst"), (1777, 64, 512, "src")])
def test_small_tiles_ragged_n(gpu_device, n, tile, interval, order):
    # activity blocks are as small as the tile when the tile is under a wave;
    # n is not a multiple of the block size
    rng = np.random.default_rng(n + tile)
    m = 6 * n
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=interval, tile=tile,
                   order=order)
    deg = np.bincount(src, minlength=n)
    for r in rmatgen.distinct_vertices(n, 3, n, eligible=deg > 0).tolist():
        say("bfs n=%d T=%d I=%d %s root=%d" % (n, tile, interval, order, r))
        ref, rounds, mx = oracle.bfs(n, src, dst, r)
        lev, st = g.bfs(r)
        assert np.array_equal(lev.cpu().numpy(), ref)
        assert st["changed_rounds"] == rounds and st["max_level"] == mx
    gs = DSSS.build(to_dev(src[: m // 8], gpu_device), to_dev(dst[: m // 8], gpu_device), n,
                    interval=interval, tile=tile, order=order, symmetrize=True)
    say("wcc n=%d T=%d I=%d %s" % (n, tile, interval, order))
    ref, rounds = oracle.wcc(n, src[: m // 8], dst[: m // 8])
    lab, st = gs.wcc()
    assert np.array_equal(lab.cpu().numpy(), ref)
    assert st["changed_rounds"] == rounds


@pytest.mark.parametrize("order", ["dst", "src"])
def test_path_streams_only_the_frontier(gpu_device, order):
    # a round streams the chunks that hold an edge out of the vertex reached in
    # the previous round: at most two chunks per round on a path
    n = 3000
    src = np.arange(n - 1, dtype=np.int32)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(src + 1, gpu_device), n, interval=128, order=order)
    lev, st = g.bfs(0)
    assert np.array_equal(lev.cpu().numpy(), np.arange(n))
    assert 0 < st["streamed_chunks"] <= 2 * st["iterations"]
    info = g.info()
    assert st["streamed_chunks"] < info["n_chunks"] * st["iterations"] // 4


@pytest.mark.parametrize("order", ["dst", "src"])
def test_edgeless_graphs(gpu_device, order):
    # no chunks at all: every round streams nothing
    import torch
    e = torch.zeros(0, dtype=torch.int32, device=gpu_device)
    g = DSSS.build(e, e, 10, interval=4, order=order)
    lev, st = g.bfs(3)
    ref = np.full(10, oracle.INF, dtype=np.int64)
    ref[3] = 0
    assert np.array_equal(lev.cpu().numpy(), ref)
    assert st["changed_rounds"] == 0 and st["max_level"] == 0 and st["streamed_chunks"] == 0
    gs = DSSS.build(e, e, 10, interval=4, order=order, symmetrize=True)
    lab, st = gs.wcc()
    assert np.array_equal(lab.cpu().numpy(), np.arange(10))
    assert st["changed_rounds"] == 0
