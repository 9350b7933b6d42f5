"""The SPU schedule with the edge stream in pinned host memory
(NXG_BUILD_HOST_STREAM, Sec. III-B1): every iteration streams the sub-shards
through two device staging buffers. Small staging buffers force many batches
and tiles split across batches; results must match the oracle to the same bars
as the device-resident runs."""
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


@pytest.mark.parametrize("order,relabel", [("dst", False), ("src", True)])
def test_fp64_fp32_against_oracle_and_device_run(gpu_device, g16, order, relabel, monkeypatch):
    src, dst, n = g16
    monkeypatch.setenv("NXG_STREAM_MB", "1")  # 1 MB buffers: a few dozen batches per iteration
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=4096, tile=8192,
                   chunk=256, order=order, relabel=relabel, host_stream=True)
    say("host stream order=%s relabel=%s words=%d" % (order, relabel, g.info()["n_words"]))
    ref, res = oracle.pagerank(n, src, dst, iters=10)
    x, st = g.pagerank(10, dtype=torch.float64)
    assert st["iterations"] == 10
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12
    x32, _ = g.pagerank(10, dtype=torch.float32)
    assert rel_l1(x32.cpu().numpy(), ref) <= 1e-5
    gd = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=4096, tile=8192,
                    chunk=256, order=order, relabel=relabel)
    xd, _ = gd.pagerank(10, dtype=torch.float64)
    assert rel_l1(x.cpu().numpy(), xd.cpu().numpy()) <= 1e-13


def test_tolerance_warm_start_weighted(gpu_device, monkeypatch):
    monkeypatch.setenv("NXG_STREAM_MB", "1")
    n = 1 << 13
    src, dst = rmatgen.rmat_edges(13, 16, seed=9)
    t = np.random.default_rng(5).random(n)
    t /= t.sum()
    w = rmatgen.row_normalized_weights(src, n, seed=109)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=1024, tile=1024,
                   chunk=256, weights=torch.from_numpy(w), keep_perm=True, host_stream=True)
    ref, res = oracle.pagerank(n, src, dst, iters=300, t=t, tol=1e-10)
    x, st = g.pagerank(300, dtype=torch.float64, tol=1e-10, teleport=torch.from_numpy(t))
    assert st["converged"] == 1 and st["iterations"] == len(res)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12
    r9, _ = oracle.pagerank(n, src, dst, iters=9)
    x4, _ = g.pagerank(4, dtype=torch.float64)
    x9, _ = g.pagerank(5, dtype=torch.float64, x0=x4)
    assert rel_l1(x9.cpu().numpy(), r9) <= 1e-12
    rw, _ = oracle.pagerank(n, src, dst, iters=12, w=w.astype(np.float64))
    xw, _ = g.pagerank(12, dtype=torch.float64, weighted=True)
    assert rel_l1(xw.cpu().numpy(), rw) <= 1e-12


def test_refusals(gpu_device):
    src, dst = rmatgen.rmat_edges(10, 8, seed=3)
    n = 1 << 10
    s, d = to_dev(src, gpu_device), to_dev(dst, gpu_device)
    w = torch.from_numpy(rmatgen.row_normalized_weights(src, n, seed=4))
    g = DSSS.build(s, d, n, weights=w, keep_perm=True, host_stream=True)
    with pytest.raises(NxgError, match="EINVAL"):
        g.bfs(0)
    with pytest.raises(NxgError, match="EINVAL"):
        g.pagerank(3, capture=True)
    with pytest.raises(NxgError, match="EINVAL"):
        g.export()
    with pytest.raises(NxgError, match="EINVAL"):
        g.set_weights(w)
    with pytest.raises(NxgError, match="EINVAL"):
        DSSS.build(s, d, n, weights=w, keep_perm=True, transpose=True, host_stream=True)
