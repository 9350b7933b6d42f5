"""Runs of equal destination in destination-ordered sub-shards are summed across
the wave before the LDS add (Sec. III-D's conflict-free reduction by
destination). These graphs put runs of every length from 1 to 70 at every lane
offset of a 64-edge slice, so runs start and end in each 16-lane row and cross
the row boundaries; PageRank (FP64), BFS and WCC are compared with the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1510_06916_amd import DSSS
from gpu_util import rel_l1, say, to_dev

pytestmark = pytest.mark.gpu


def run_graph(n, lengths, seed):
    # destination v (in increasing order) receives lengths[v] edges from
    # distinct sources; in destination order they form one run per destination
    rng = np.random.default_rng(seed)
    src, dst = [], []
    for v, k in enumerate(lengths):
        s = rng.choice(n, size=k, replace=False)
        src.append(s)
        dst.append(np.full(k, v))
    src = np.concatenate(src).astype(np.int32)
    dst = np.concatenate(dst).astype(np.int32)
    return src, dst


@pytest.mark.parametrize("shift", [0, 1, 5, 17, 33])
def test_runs_of_every_length(gpu_device, shift):
    n = 4096
    # a leading block of single edges moves every later run to another lane offset
    lengths = [1] * shift + [k for k in range(1, 71)] + [64, 63, 65, 128, 200, 1, 2, 3] * 4
    lengths += [0] * (n - len(lengths))
    src, dst = run_graph(n, lengths, seed=100 + shift)
    say("runs graph shift=%d m=%d" % (shift, len(src)))
    # one interval and one tile: the stream is exactly the destination-sorted list
    kw = dict(interval=n, tile=n, chunk=256, order="dst")
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, value_bytes=8, **kw)
    x, _ = g.pagerank(6, dtype=torch.float64)
    ref, _ = oracle.pagerank(n, src, dst, iters=6)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12
    # several intervals: runs broken by interval markers, same destinations again
    g2 = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, value_bytes=8, interval=700,
                    tile=n, chunk=256, order="dst")
    x2, _ = g2.pagerank(6, dtype=torch.float64)
    assert rel_l1(x2.cpu().numpy(), ref) <= 1e-12
    # minimum programs take the same path with their own identity
    gb = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, value_bytes=4, **kw)
    for root in (int(src[0]), int(src[len(src) // 2])):
        lev, st = gb.bfs(root)
        rl, rounds, mx = oracle.bfs(n, src, dst, root)
        assert np.array_equal(lev.cpu().numpy(), rl) and st["max_level"] == mx
    gw = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, value_bytes=4, symmetrize=True, **kw)
    lab, _ = gw.wcc()
    rw, _ = oracle.wcc(n, src, dst)
    assert np.array_equal(lab.cpu().numpy(), rw)
