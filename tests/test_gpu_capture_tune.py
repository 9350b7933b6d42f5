"""hipGraph capture of PageRank runs (replays checked against eager runs) and the
autotuner (valid layouts, cache file)."""
import numpy as np
import pytest
import torch

import oracle
import rmatgen
from paper_1510_06916_amd import DSSS, tune
from gpu_util import rel_l1, say, to_dev

pytestmark = pytest.mark.gpu


def test_capture_replays_match_eager(gpu_device):
    n = 1 << 13
    src, dst = rmatgen.rmat_edges(13, 8, seed=90)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=1024, tile=2048)
    ref, _ = oracle.pagerank(n, src, dst, iters=12)
    eager, _ = g.pagerank(12, dtype=torch.float64)
    out = torch.empty(n, dtype=torch.float64, device=gpu_device)
    for rep in range(4):
        out.fill_(-1.0)
        x, st = g.pagerank(12, dtype=torch.float64, capture=True, out=out)
        assert x.data_ptr() == out.data_ptr() and st["iterations"] == 12
        say("replay %d: rel-L1 vs eager %.2e" % (rep, rel_l1(x.cpu().numpy(), eager.cpu().numpy())))
        assert rel_l1(x.cpu().numpy(), eager.cpu().numpy()) <= 1e-13
        assert rel_l1(x.cpu().numpy(), ref) <= 1e-12
        # eager work and a sync between replays
        g.pagerank(3, dtype=torch.float32)
        torch.cuda.synchronize()


def test_capture_weighted_fp32(gpu_device):
    n = 1 << 12
    src, dst = rmatgen.rmat_edges(12, 8, seed=91)
    w = rmatgen.row_normalized_weights(src, n, seed=191)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=512,
                   weights=torch.from_numpy(w))
    ref, _ = oracle.pagerank(n, src, dst, iters=9, w=w.astype(np.float64))
    out = torch.empty(n, dtype=torch.float32, device=gpu_device)
    for _ in range(3):
        x, _ = g.pagerank(9, dtype=torch.float32, weighted=True, capture=True, out=out)
        assert rel_l1(x.cpu().numpy(), ref) <= 1e-5


def test_capture_rejects_tolerance(gpu_device):
    src, dst = rmatgen.rmat_edges(8, 4, seed=1)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), 256)
    with pytest.raises(Exception, match="EINVAL"):
        g.pagerank(5, tol=1e-6, capture=True)


def test_tune_picks_a_valid_layout_and_caches(gpu_device, tmp_path, monkeypatch):
    monkeypatch.setenv("NXG_TUNE_CACHE", str(tmp_path / "tune.txt"))
    n = 1 << 14
    src, dst = rmatgen.rmat_edges(14, 8, seed=92)
    s, d = to_dev(src, gpu_device), to_dev(dst, gpu_device)
    r = tune(s, d, n)
    say("tune: %s" % r)
    assert r["candidates"] > 4 and r["ms_per_iter"] > 0
    assert r["interval"] >= 1 and r["tile"] >= 1 and r["chunk"] in (512, 1024, 2048)
    assert r["order"] in (0, 1) and r["relabel"] in (0, 1)
    r2 = tune(s, d, n)
    assert r2["candidates"] == 0 and r2["interval"] == r["interval"]
    assert r2["order"] == r["order"] and r2["relabel"] == r["relabel"]
    assert (tmp_path / "tune.txt").read_text().count("|") == 1
    assert r["width"] == 1 and r["pairs"] in (0, 1)
    g = DSSS.build(s, d, n, interval=r["interval"], tile=r["tile"], chunk=r["chunk"],
                   order=("dst", "src")[r["order"]], relabel=bool(r["relabel"]), pairs=bool(r["pairs"]))
    x, _ = g.pagerank(10, dtype=torch.float32, piece_chunks=r["piece_chunks"])
    ref, _ = oracle.pagerank(n, src, dst, iters=10)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("batch", [40, 8])
def test_tune_batched_width(gpu_device, tmp_path, monkeypatch, batch):
    # the batched tuner picks a vector width and a layout; running the batch
    # in passes of that width matches plain single-seed runs
    monkeypatch.setenv("NXG_TUNE_CACHE", str(tmp_path / "tune.txt"))
    n = 1 << 13
    src, dst = rmatgen.rmat_edges(13, 8, seed=93)
    s, d = to_dev(src, gpu_device), to_dev(dst, gpu_device)
    r = tune(s, d, n, batch=batch)
    say("batched tune (batch %d): %s" % (batch, r))
    widths = [min(batch, 64)] + [w for w in (32, 16) if w < min(batch, 64)]
    assert r["width"] in widths and r["candidates"] >= len(widths) and r["ms_per_iter"] > 0
    r2 = tune(s, d, n, batch=batch)
    assert r2["candidates"] == 0 and r2["width"] == r["width"] and r2["tile"] == r["tile"]
    w = r["width"]
    g = DSSS.build(s, d, n, interval=r["interval"], tile=r["tile"], chunk=r["chunk"],
                   order=("dst", "src")[r["order"]], relabel=bool(r["relabel"]), value_bytes=8 * w)
    seeds = torch.from_numpy(rmatgen.distinct_vertices(94, batch, n))
    cols = torch.cat([g.ppr(seeds[i:i + w], 12)[0] for i in range(0, batch, w)], dim=1)
    assert cols.shape == (n, batch)
    gp = DSSS.build(s, d, n)
    for b in (0, batch - 1):
        tele = torch.zeros(n, dtype=torch.float32, device=gpu_device)
        tele[int(seeds[b])] = 1.0
        xp, _ = gp.pagerank(12, dtype=torch.float32, teleport=tele)
        assert rel_l1(cols[:, b].cpu().numpy(), xp.cpu().numpy()) <= 1e-6
