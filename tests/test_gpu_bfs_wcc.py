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
