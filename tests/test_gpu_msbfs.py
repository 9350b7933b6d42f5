"""Several BFS at once (one 64-bit root set per vertex) against the oracle's
BFS from each root, bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import rmatgen
from paper_1510_06916_amd import DSSS, _lib
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def _check(g, n, src, dst, roots, what):
    say("multi-root bfs " + what)
    lev, st = g.bfs_multi(roots)
    lev = lev.cpu().numpy()
    assert lev.shape == (n, len(roots))
    deg = np.bincount(src, minlength=n)
    reached, mx = 0, 0
    for b, r in enumerate(roots):
        ref, rounds, m = oracle.bfs(n, src, dst, r)
        assert np.array_equal(lev[:, b], ref), (what, b, r)
        reached += int(deg[ref != oracle.INF].sum())
        mx = max(mx, m)
    assert st["max_level"] == mx and st["changed_rounds"] == mx
    assert st["reached_edges"] == reached
    return st


@pytest.mark.parametrize("scale,B,interval,tile,order,relabel", [
    (12, 2, 512, 0, "dst", False), (14, 16, 1000, 0, "dst", False), (14, 64, 2048, 4096, "src", True),
    (13, 33, 1024, 8192, "dst", True), (15, 16, 4096, 0, "src", False)])
def test_msbfs_rmat(gpu_device, scale, B, interval, tile, order, relabel):
    n = 1 << scale
    src, dst = rmatgen.rmat_edges(scale, 8, seed=scale + 30)
    deg = np.bincount(src, minlength=n)
    roots = rmatgen.distinct_vertices(scale + 130, B - 1, n, eligible=deg > 0).tolist()
    roots.append(int(np.flatnonzero(deg == 0)[0]))  # a root with no out-edges
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=interval, tile=tile,
                   order=order, relabel=relabel, value_bytes=8)
    _check(g, n, src, dst, roots, "scale=%d B=%d I=%d %s relabel=%s" % (scale, B, interval, order, relabel))
    # the same roots again on the same handle, and repeated roots
    _check(g, n, src, dst, roots[:2] + roots[:2], "repeated roots")


def test_msbfs_degree_split_tiles_path(gpu_device, monkeypatch):
    # pieces of 2 chunks split the tiles; degreeing drops ids without edges, one
    # of which is a root (it reaches only itself)
    monkeypatch.setenv("NXG_PIECE_CHUNKS", "2")
    n = 40000
    rs, rd = rmatgen.rmat_edges(15, 8, seed=61)
    src = np.concatenate([rs, 30000 + np.arange(5000)]).astype(np.int32)
    dst = np.concatenate([rd, 30001 + np.arange(5000)]).astype(np.int32)  # a long path
    used = np.zeros(n, bool)
    used[src] = used[dst] = True
    dropped = int(np.flatnonzero(~used)[0])
    roots = [0, 30000, dropped, 5, 31234, 17]
    for order, relabel, degree in (("dst", False, False), ("src", True, True)):
        g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=3000, tile=4096, chunk=256,
                       order=order, relabel=relabel, degree=degree, value_bytes=8)
        _check(g, n, src, dst, roots, "path %s relabel=%s degree=%s" % (order, relabel, degree))


def test_msbfs_refusals(gpu_device):
    n = 1 << 16
    src, dst = rmatgen.rmat_edges(16, 4, seed=5)
    g4 = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=4096, tile=32768,
                    value_bytes=4)
    with pytest.raises(_lib.NxgError) as e:
        g4.bfs_multi([1, 2])   # 4-byte tile too large for 8-byte root sets
    assert e.value.status == _lib.NXG_EINVAL
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=4096, value_bytes=8)
    with pytest.raises(_lib.NxgError):
        g.bfs_multi([1, n])    # root out of range
    with pytest.raises(_lib.NxgError):
        g.bfs_multi(list(range(65)))
    lev, st = g.bfs_multi([0, 1], max_rounds=1)
    assert st["status"] in (_lib.NXG_OK, _lib.NXG_ENOTCONV)


def test_msbfs_empty_graph(gpu_device):
    e = torch.zeros(0, dtype=torch.int32, device=gpu_device)
    n = 50
    g = DSSS.build(e, e, n, interval=16, value_bytes=8)
    roots = [3, 49, 3]
    lev, st = g.bfs_multi(roots)
    lev = lev.cpu().numpy()
    want = np.full((n, 3), oracle.INF, dtype=np.int32)
    for b, r in enumerate(roots):
        want[r, b] = 0
    assert np.array_equal(lev, want) and st["max_level"] == 0 and st["reached_edges"] == 0
