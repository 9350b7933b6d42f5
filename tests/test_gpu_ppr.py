"""Batched personalised PageRank ([n, B] values) against single-seed plain runs and
the FP64 oracle; superposition across columns."""
import numpy as np
import pytest
import torch

import oracle
import rmatgen
from paper_1510_06916_amd import DSSS
from gpu_util import rel_l1, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("scale,B,tile,interval", [(12, 64, 256, 1024), (13, 17, 512, 2048),
                                                   (12, 1, 4096, 4096), (12, 64, 128, 300)])
def test_batched_matches_plain_and_oracle(gpu_device, scale, B, tile, interval):
    n = 1 << scale
    src, dst = rmatgen.rmat_edges(scale, 8, seed=scale + 400)
    seeds = rmatgen.distinct_vertices(scale + 104, B, n)
    say("ppr scale=%d B=%d tile=%d I=%d" % (scale, B, tile, interval))
    gb = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=interval,
                    tile=tile, value_bytes=8 * B)
    xb, st = gb.ppr(torch.from_numpy(seeds), 30)
    assert xb.shape == (n, B) and st["iterations"] == 30
    xb = xb.cpu().numpy().astype(np.float64)
    gp = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=interval)
    for b in sorted(set([0, B // 2, B - 1])):
        t = np.zeros(n)
        t[seeds[b]] = 1.0
        xp, _ = gp.pagerank(30, dtype=torch.float32, teleport=torch.from_numpy(t))
        ref, _ = oracle.pagerank(n, src, dst, iters=30, t=t)
        assert rel_l1(xb[:, b], xp.cpu().numpy()) <= 1e-6
        assert rel_l1(xb[:, b], ref) <= 1e-5
    assert np.allclose(xb.sum(0), 1.0, atol=1e-5)


def test_batched_tolerance_stop(gpu_device):
    n = 1 << 11
    src, dst = rmatgen.rmat_edges(11, 8, seed=3)
    seeds = np.arange(8, dtype=np.int32) * 7
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=512, tile=512,
                   value_bytes=64)
    x, st = g.ppr(torch.from_numpy(seeds), 500, tol=1e-6)
    assert st["converged"] == 1 and st["iterations"] < 500
    t = np.zeros(n)
    t[seeds[3]] = 1.0
    ref, res = oracle.pagerank(n, src, dst, iters=500, t=t, tol=1e-9)
    assert rel_l1(x[:, 3].cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("relabel", [False, True])
def test_batched_capture_replays(gpu_device, relabel):
    # a captured batched run replays against eager runs, also after the seed
    # buffer's contents change (the graph reads the seeds at every replay)
    scale, B, iters = 12, 32, 9
    n = 1 << scale
    src, dst = rmatgen.rmat_edges(scale, 8, seed=scale + 40)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=1024, tile=512,
                   value_bytes=8 * B, relabel=relabel)
    seeds = to_dev(rmatgen.distinct_vertices(61, B, n), gpu_device)
    out = torch.empty((n, B), dtype=torch.float32, device=gpu_device)
    for rep in range(3):
        if rep == 2:
            seeds.copy_(to_dev(rmatgen.distinct_vertices(62, B, n), gpu_device))
        say("ppr capture relabel=%d replay %d" % (relabel, rep))
        g.ppr(seeds, iters, out=out, capture=True)
        xe, _ = g.ppr(seeds.clone(), iters)
        torch.cuda.synchronize()
        for b in range(B):
            assert rel_l1(out[:, b].cpu().numpy(), xe[:, b].cpu().numpy()) <= 1e-6
