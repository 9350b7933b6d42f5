"""PageRank on the GPU against the FP64 oracle (FP64 <= 1e-12, FP32 <= 1e-5 rel. L1)."""
import os

import numpy as np
import pytest
import torch

import oracle
import rmatgen
from paper_1510_06916_amd import DSSS
from gpu_util import rel_l1, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfg1(gpu_device):
    # R-MAT scale 16, edge factor 16, seed 1, 4 intervals: the FP64 parity config
    src, dst = rmatgen.rmat_edges(16, 16, seed=1)
    return src, dst, 1 << 16


def test_cfg1_fp64_10_iterations(gpu_device, cfg1):
    src, dst, n = cfg1
    say("cfg1 fp64: n=%d m=%d P=4" % (n, len(src)))
    ref, res = oracle.pagerank(n, src, dst, iters=10)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, P=4, value_bytes=8)
    x, st = g.pagerank(10, dtype=torch.float64)
    x = x.cpu().numpy()
    assert rel_l1(x, ref) <= 1e-12
    assert abs(x.sum() - 1.0) < 1e-12
    assert st["iterations"] == 10


@pytest.mark.parametrize("piece", ["1", "3", "1000000"])
def test_cfg1_fp32_piece_sizes(gpu_device, cfg1, piece, monkeypatch):
    src, dst, n = cfg1
    monkeypatch.setenv("NXG_PIECE_CHUNKS", piece)
    ref, _ = oracle.pagerank(n, src, dst, iters=10)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, P=4)
    say("cfg1 fp32 piece=%s" % piece)
    x, st = g.pagerank(10, dtype=torch.float32)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("interval,tile,chunk,order", [
    (4096, 0, 256, "dst"), (1000, 256, 256, "dst"), (65536, 2048, 1024, "dst"),
    (2048, 16384, 256, "dst"), (3000, 8192, 1024, "dst"), (4096, 16384, 1024, "src"),
    (16384, 16384, 2048, "src")])
def test_layouts_fp64(gpu_device, cfg1, interval, tile, chunk, order):
    src, dst, n = cfg1
    ref, _ = oracle.pagerank(n, src, dst, iters=6)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=interval,
                   tile=tile, chunk=chunk, value_bytes=8, order=order)
    say("layout I=%d tile=%d chunk=%d order=%s" % (interval, tile, chunk, order))
    x, _ = g.pagerank(6, dtype=torch.float64)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12


def test_teleport_tolerance_and_warm_start(gpu_device):
    n = 1 << 12
    src, dst = rmatgen.rmat_edges(12, 8, seed=7)
    rng = np.random.default_rng(5)
    t = rng.random(n)
    t /= t.sum()
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=1024,
                   value_bytes=8)
    ref, res = oracle.pagerank(n, src, dst, iters=200, t=t, tol=1e-10)
    x, st = g.pagerank(200, dtype=torch.float64, tol=1e-10, teleport=torch.from_numpy(t))
    say("tol run: oracle %d its, gpu %d its" % (len(res), st["iterations"]))
    assert st["converged"] == 1 and st["iterations"] == len(res)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12
    # 7 iterations then 5 more from that vector == 12 iterations
    r12, _ = oracle.pagerank(n, src, dst, iters=12, t=t)
    x7, _ = g.pagerank(7, dtype=torch.float64, teleport=torch.from_numpy(t))
    x12, _ = g.pagerank(5, dtype=torch.float64, teleport=torch.from_numpy(t), x0=x7)
    assert rel_l1(x12.cpu().numpy(), r12) <= 1e-12
    # not converged within max_iters -> ENOTCONV, values still written
    x3, st3 = g.pagerank(3, dtype=torch.float64, tol=1e-14)
    assert st3["status"] == 4 and st3["converged"] == 0
    r3, _ = oracle.pagerank(n, src, dst, iters=3)
    assert rel_l1(x3.cpu().numpy(), r3) <= 1e-12


def test_weighted_fp64(gpu_device):
    n = 1 << 12
    src, dst = rmatgen.rmat_edges(12, 8, seed=8)
    w = rmatgen.row_normalized_weights(src, n, seed=108)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=512,
                   weights=torch.from_numpy(w), value_bytes=8)
    ref, _ = oracle.pagerank(n, src, dst, iters=15, w=w.astype(np.float64))
    x, _ = g.pagerank(15, dtype=torch.float64, weighted=True)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12


@pytest.mark.parametrize("order,relabel", [("dst", False), ("src", True)])
def test_extreme_hub_ragged_n_many_pieces(gpu_device, order, relabel, monkeypatch):
    # every vertex points at vertex 7 (one tile holds a fifth of the edges), plus
    # R-MAT edges; n is not a multiple of any tile or interval; pieces of 2
    # chunks force hundreds of hub slots and finishing segments
    n = 100003
    rs, rd = rmatgen.rmat_edges(16, 8, seed=41)
    rs, rd = rs % n, rd % n
    hub_s = np.arange(n, dtype=np.int64)
    src = np.concatenate([rs, hub_s]).astype(np.int32)
    dst = np.concatenate([rd, np.full(n, 7)]).astype(np.int32)
    key = np.unique(src.astype(np.int64) * n + dst)
    src, dst = (key // n).astype(np.int32), (key % n).astype(np.int32)
    ref, _ = oracle.pagerank(n, src, dst, iters=8)
    monkeypatch.setenv("NXG_PIECE_CHUNKS", "2")
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=3000, tile=4096,
                   chunk=256, order=order, relabel=relabel)
    say("hub graph n=%d m=%d order=%s relabel=%s" % (n, len(src), order, relabel))
    x, _ = g.pagerank(8, dtype=torch.float64)
    # the hub sums ~1e5 terms in FP64 in another order than the oracle: the
    # worst-case rounding of such a sum is k*u ~ 1e5 * 1.1e-16 ~ 1e-11 relative,
    # and the hub carries most of the L1 mass, so the FP64 bar here is 1e-11
    # (a lost or doubled piece would show as ~1e-3)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-11
    x32, _ = g.pagerank(8, dtype=torch.float32)
    assert rel_l1(x32.cpu().numpy(), ref) <= 1e-5
    gb = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=3000, tile=4096,
                    chunk=256, value_bytes=4, order=order, relabel=relabel)
    lev, st = gb.bfs(3)
    rl, rounds, mx = oracle.bfs(n, src, dst, 3)
    assert np.array_equal(lev.cpu().numpy(), rl) and st["max_level"] == mx
