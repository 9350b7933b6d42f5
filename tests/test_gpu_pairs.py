"""The pair layout (NXG_BUILD_PAIRS: two destinations of one source per word,
under a header word naming the source) against the FP64 oracle; the plain
source-order layout of the same graph is the comparison for the word count."""
import numpy as np
import pytest
import torch

import oracle
import rmatgen
from paper_1510_06916_amd import DSSS, NxgError
from gpu_util import rel_l1, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rmat14(gpu_device):
    src, dst = rmatgen.rmat_edges(14, 16, seed=14)
    return src, dst, 1 << 14


@pytest.mark.parametrize("interval,tile,chunk,relabel", [
    (2048, 16384, 256, True), (2048, 16384, 1024, False), (1000, 256, 256, True),
    (4096, 2048, 512, False), (16384, 16384, 2048, True), (512, 64, 256, True)])
def test_fp64_and_fp32(gpu_device, rmat14, interval, tile, chunk, relabel):
    src, dst, n = rmat14
    ref, _ = oracle.pagerank(n, src, dst, iters=8)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=interval, tile=tile,
                   chunk=chunk, order="src", relabel=relabel, pairs=True)
    plain = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=interval,
                       tile=tile, chunk=chunk, order="src", relabel=relabel)
    info = g.info()
    say("pairs I=%d T=%d C=%d relabel=%d: %d words vs %d" % (interval, tile, chunk, relabel,
                                                           info["n_words"], plain.info()["n_words"]))
    assert info["pairs"] == 1 and info["m"] == len(src)
    assert info["n_words"] <= plain.info()["n_words"]
    x, st = g.pagerank(8, dtype=torch.float64)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12
    x32, _ = g.pagerank(8, dtype=torch.float32)
    assert rel_l1(x32.cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("piece", [1, 3])
def test_split_tiles_capture_tolerance(gpu_device, rmat14, piece):
    # hub runs split over chunks and pieces; a captured replay; a tolerance stop
    src, dst, n = rmat14
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=1024, tile=4096,
                   chunk=256, order="src", relabel=True, pairs=True)
    ref, _ = oracle.pagerank(n, src, dst, iters=12)
    x, _ = g.pagerank(12, dtype=torch.float64, piece_chunks=piece)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12
    for _ in range(2):
        xc, _ = g.pagerank(12, dtype=torch.float64, capture=True, piece_chunks=piece)
        torch.cuda.synchronize()
        assert rel_l1(xc.cpu().numpy(), ref) <= 1e-12
    xt, st = g.pagerank(500, dtype=torch.float64, tol=1e-10, piece_chunks=piece)
    assert st["residual"] <= 1e-10 and st["iterations"] < 500
    fix, _ = oracle.pagerank(n, src, dst, iters=st["iterations"])
    assert rel_l1(xt.cpu().numpy(), fix) <= 1e-12


def test_star_runs_and_ragged_n(gpu_device):
    # one source with edges to every vertex (runs of every length and parity),
    # a cycle, duplicate edges, n not a power of two
    n = 3001
    rng = np.random.default_rng(7)
    hub = np.zeros(n, dtype=np.int32)
    cyc = np.arange(n, dtype=np.int32)
    extra = rng.integers(0, n, 4 * n).astype(np.int32)
    src = np.concatenate([hub, cyc, extra[: 2 * n], np.full(5, 17, np.int32)])
    dst = np.concatenate([np.arange(n, dtype=np.int32), (cyc + 1) % n, extra[2 * n:],
                          np.full(5, 99, np.int32)])
    ref, _ = oracle.pagerank(n, src, dst, iters=7)
    for tile, interval in ((1024, 256), (16384, 2048), (128, 1024)):
        g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=interval,
                       tile=tile, chunk=256, order="src", pairs=True)
        say("star n=%d T=%d I=%d" % (n, tile, interval))
        x, _ = g.pagerank(7, dtype=torch.float64)
        assert rel_l1(x.cpu().numpy(), ref) <= 1e-12


def test_refusals(gpu_device):
    src = to_dev(np.array([0, 1, 2], dtype=np.int32), gpu_device)
    dst = to_dev(np.array([1, 2, 0], dtype=np.int32), gpu_device)
    with pytest.raises(NxgError, match="EINVAL"):
        DSSS.build(src, dst, 3, pairs=True)  # destination order
    with pytest.raises(NxgError, match="EINVAL"):  # a tile of 32768 vertices
        DSSS.build(src, dst, 40000, order="src", tile=32768, value_bytes=4, pairs=True)
    with pytest.raises(NxgError, match="EINVAL"):
        DSSS.build(src, dst, 3, order="src", pairs=True, weights=torch.ones(3))
    with pytest.raises(NxgError, match="EINVAL"):
        DSSS.build(src, dst, 3, order="src", pairs=True, symmetrize=True)
    g = DSSS.build(src, dst, 3, order="src", pairs=True)
    with pytest.raises(NxgError, match="EINVAL"):
        g.bfs(0)
    with pytest.raises(NxgError, match="EINVAL"):
        g.export()
    x, _ = g.pagerank(5, dtype=torch.float64)
    assert torch.allclose(x.cpu(), torch.full((3,), 1.0 / 3, dtype=torch.float64), atol=1e-15)
