"""The coarse-grained, source-sorted comparison scheme (NXG_BUILD_SCATTER +
NXG_RUN_SCATTER, Sec. IV-B1): the whole edge list in (source, destination) order,
pushed into global FP64 sums with atomics, against the FP64 oracle to the same bars
as the DSSS runs (FP64 <= 1e-12, FP32 <= 1e-5 relative L1)."""
import numpy as np
import pytest
import torch

import oracle
import rmatgen
from paper_1510_06916_amd import DSSS, NxgError
from gpu_util import rel_l1, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g16(gpu_device):
    src, dst = rmatgen.rmat_edges(16, 16, seed=1)
    return src, dst, 1 << 16


def test_layout_is_the_source_sorted_edge_list(gpu_device):
    src, dst = rmatgen.rmat_edges(12, 8, seed=31)
    n = 3000  # ragged: not a power of two; ids folded into range
    src, dst = (src % n).astype(np.int32), (dst % n).astype(np.int32)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, scatter=True)
    inf = g.info()
    assert inf["n_tiles"] == 1 and inf["order"] == 1 and inf["tile"] >= n
    assert inf["interval"] <= 1 << (31 - int(np.ceil(np.log2(n))))
    ex = g.export()
    o = np.lexsort((dst, src))
    assert np.array_equal(ex["src"].cpu().numpy(), src[o])
    assert np.array_equal(ex["dst"].cpu().numpy(), dst[o])


def test_fp64_and_fp32(gpu_device, g16):
    src, dst, n = g16
    ref, res = oracle.pagerank(n, src, dst, iters=10)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, scatter=True)
    say("scatter fp64/fp32 n=%d m=%d I=%d" % (n, len(src), g.info()["interval"]))
    x, st = g.pagerank(10, dtype=torch.float64, scatter=True)
    assert st["iterations"] == 10
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12
    assert abs(st["residual"] - res[-1]) <= 1e-12 + 1e-9 * res[-1]
    x32, _ = g.pagerank(10, dtype=torch.float32, scatter=True)
    assert rel_l1(x32.cpu().numpy(), ref) <= 1e-5
    # the DSSS run of the same graph agrees to the order of the additions
    gd = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n)
    xd, _ = gd.pagerank(10, dtype=torch.float64)
    assert rel_l1(x.cpu().numpy(), xd.cpu().numpy()) <= 1e-13


def test_small_intervals_teleport_tolerance_warm_start(gpu_device):
    src, dst = rmatgen.rmat_edges(12, 8, seed=7)
    n = 1 << 12
    rng = np.random.default_rng(5)
    t = rng.random(n)
    t /= t.sum()
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=64, chunk=256,
                   scatter=True)
    assert g.info()["interval"] == 64
    ref, res = oracle.pagerank(n, src, dst, iters=200, t=t, tol=1e-10)
    x, st = g.pagerank(200, dtype=torch.float64, tol=1e-10, teleport=torch.from_numpy(t), scatter=True)
    assert st["converged"] == 1 and st["iterations"] == len(res)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12
    r12, _ = oracle.pagerank(n, src, dst, iters=12, t=t)
    x7, _ = g.pagerank(7, dtype=torch.float64, teleport=torch.from_numpy(t), scatter=True)
    x12, _ = g.pagerank(5, dtype=torch.float64, teleport=torch.from_numpy(t), x0=x7, scatter=True)
    assert rel_l1(x12.cpu().numpy(), r12) <= 1e-12
    x0, st0 = g.pagerank(0, dtype=torch.float64, teleport=torch.from_numpy(t), scatter=True)
    assert st0["iterations"] == 0 and np.allclose(x0.cpu().numpy(), t, rtol=0, atol=1e-18)


def test_weighted(gpu_device):
    src, dst = rmatgen.rmat_edges(12, 8, seed=17)
    n = 1 << 12
    w = rmatgen.row_normalized_weights(src, n, seed=33)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, weights=torch.from_numpy(w),
                   keep_perm=True, scatter=True)
    ref, _ = oracle.pagerank(n, src, dst, iters=15, w=w.astype(np.float64))
    x, _ = g.pagerank(15, dtype=torch.float64, weighted=True, scatter=True)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12


def test_degenerate_graphs(gpu_device):
    # no edges: every vertex dangling, x stays uniform; one vertex with a self-loop
    e = np.zeros(0, np.int32)
    g = DSSS.build(to_dev(e, gpu_device), to_dev(e, gpu_device), 100, scatter=True)
    x, _ = g.pagerank(5, dtype=torch.float64, scatter=True)
    assert np.allclose(x.cpu().numpy(), 0.01, rtol=0, atol=1e-15)
    one = np.zeros(1, np.int32)
    g1 = DSSS.build(to_dev(one, gpu_device), to_dev(one, gpu_device), 1, scatter=True)
    x1, _ = g1.pagerank(3, dtype=torch.float64, scatter=True)
    assert abs(float(x1.cpu()[0]) - 1.0) <= 1e-15


def test_refusals(gpu_device, g16):
    src, dst, n = g16
    s, d = to_dev(src, gpu_device), to_dev(dst, gpu_device)
    gs = DSSS.build(s, d, n, scatter=True)
    with pytest.raises(NxgError, match="EINVAL"):
        gs.pagerank(3)  # DSSS run on the scatter layout
    with pytest.raises(NxgError, match="EINVAL"):
        gs.bfs(0)
    with pytest.raises(NxgError, match="EINVAL"):
        gs.pagerank(3, scatter=True, capture=True)
    gd = DSSS.build(s, d, n)
    with pytest.raises(NxgError, match="EINVAL"):
        gd.pagerank(3, scatter=True)  # scatter run on a DSSS layout
    with pytest.raises(NxgError, match="EINVAL"):
        DSSS.build(s, d, n, scatter=True, relabel=True)
