"""DSSS construction on the GPU against the oracle's DSSS order (bit-exact)."""
import numpy as np
import pytest
import torch

import oracle
import rmatgen
from paper_1510_06916_amd import DSSS, NxgError
from test_oracle_dsss import load_fig1
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def _stream_order(src, dst, I, T, order="dst"):
    """(tile, source interval, dst, src) order -- (tile, interval, src, dst) for the
    source-major ablation; with T == I and order "dst" this is the DSSS order."""
    tau = dst // T
    idx = np.arange(len(src))
    if order == "dst":
        return np.lexsort((idx, src, dst, src // I, tau))
    return np.lexsort((idx, dst, src, src // I, tau))


def test_paper_example(gpu_device):
    meta, want = load_fig1()
    edges = want + [(0, 1), (1, 0), (2, 5), (3, 5), (6, 7), (7, 2), (4, 4), (5, 0), (0, 3)]
    order = np.random.default_rng(0).permutation(len(edges))
    src = np.array([edges[k][0] for k in order], np.int32)
    dst = np.array([edges[k][1] for k in order], np.int32)
    say("paper example: n=8 I=2")
    # tile == interval makes the stream order exactly the paper's DSSS order
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), 8,
                   interval=meta["interval_size"], tile=meta["interval_size"], keep_perm=True)
    ex = g.export(perm=True)
    off = ex["offsets"].cpu().numpy()
    P = 4
    s = meta["destination_interval"] * P + meta["source_interval"]
    es, ed = ex["src"].cpu().numpy(), ex["dst"].cpu().numpy()
    assert list(zip(es[off[s]:off[s + 1]].tolist(), ed[off[s]:off[s + 1]].tolist())) == want
    perm_o, off_o = oracle.dsss_order(8, src, dst, meta["interval_size"])
    assert np.array_equal(off, off_o)
    assert np.array_equal(ex["perm"].cpu().numpy(), perm_o)


@pytest.mark.parametrize("n,interval,tile,chunk,order", [
    (1000, 250, 256, 256, "dst"), (1000, 64, 0, 256, "dst"), (1000, 1, 0, 256, "dst"),
    (1000, 1000, 1024, 512, "dst"), (4096, 1024, 256, 256, "dst"), (5000, 3000, 1024, 1024, "dst"),
    (4096, 4096, 64, 256, "dst"), (77, 7, 0, 256, "dst"), (4096, 512, 4096, 256, "dst"),
    (5000, 700, 2048, 256, "dst"), (4096, 1024, 1024, 256, "src"), (5000, 300, 4096, 512, "src"),
])
def test_structure_matches_oracle(gpu_device, n, interval, tile, chunk, order):
    src, dst = rmatgen.rmat_edges(13, 8, seed=12)
    keep = (src < n) & (dst < n)
    src, dst = src[keep], dst[keep]
    rng = np.random.default_rng(n + interval)
    dup = rng.choice(len(src), min(50, len(src)), replace=False)
    src = np.concatenate([src, src[dup]]).astype(np.int32)
    dst = np.concatenate([dst, dst[dup]]).astype(np.int32)
    p = rng.permutation(len(src))
    src, dst = src[p], dst[p]
    say("build n=%d I=%d tile=%d chunk=%d order=%s m=%d" % (n, interval, tile, chunk, order,
                                                            len(src)))
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=interval,
                   tile=tile, chunk=chunk, keep_perm=True, order=order)
    inf = g.info()
    assert inf["m"] == len(src) and inf["P"] == -(-n // interval)
    ex = g.export(perm=True)
    perm_o, off_o = oracle.dsss_order(n, src, dst, interval)
    assert np.array_equal(ex["offsets"].cpu().numpy(), off_o)
    want = _stream_order(src.astype(np.int64), dst.astype(np.int64), interval, inf["tile"], order)
    assert np.array_equal(ex["perm"].cpu().numpy(), want)
    assert np.array_equal(ex["src"].cpu().numpy(), src[want])
    assert np.array_equal(ex["dst"].cpu().numpy(), dst[want])
    if inf["tile"] == interval and order == "dst":
        assert np.array_equal(want, perm_o)


def test_dedup_and_symmetrize(gpu_device):
    src, dst = rmatgen.rmat_edges(10, 8, seed=3)
    src2 = np.concatenate([src, src[:100]]).astype(np.int32)
    dst2 = np.concatenate([dst, dst[:100]]).astype(np.int32)
    g = DSSS.build(to_dev(src2, gpu_device), to_dev(dst2, gpu_device), 1024, interval=128,
                   dedup=True)
    assert g.m == len(src)
    gs = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), 1024, interval=128,
                    symmetrize=True)
    keys = np.unique(np.concatenate([src.astype(np.int64) * 1024 + dst,
                                     dst.astype(np.int64) * 1024 + src]))
    assert gs.m == len(keys)
    ex = gs.export()
    got = np.sort(ex["src"].cpu().numpy().astype(np.int64) * 1024 + ex["dst"].cpu().numpy())
    assert np.array_equal(got, keys)


def test_invalid_ids_rejected(gpu_device):
    src = torch.tensor([0, 1, 5], dtype=torch.int32, device=gpu_device)
    dst = torch.tensor([1, 2, 0], dtype=torch.int32, device=gpu_device)
    with pytest.raises(NxgError, match="EINVAL"):
        DSSS.build(src, dst, 5)
    with pytest.raises(NxgError, match="EINVAL"):
        DSSS.build(src, dst - 1, 6)


def test_empty_graph_and_single_vertex(gpu_device):
    e = torch.zeros(0, dtype=torch.int32, device=gpu_device)
    g = DSSS.build(e, e, 10, interval=4)
    assert g.m == 0
    x, st = g.pagerank(5, dtype=torch.float64)
    assert torch.allclose(x, torch.full_like(x, 0.1), atol=1e-15)
    g1 = DSSS.build(torch.zeros(1, dtype=torch.int32, device=gpu_device),
                    torch.zeros(1, dtype=torch.int32, device=gpu_device), 1)
    x, _ = g1.pagerank(3, dtype=torch.float64)
    assert abs(float(x[0]) - 1.0) < 1e-15
    lev, st = g1.bfs(0)
    assert lev.tolist() == [0]


def test_bandwidth_probes(gpu_device):
    from paper_1510_06916_amd import copy_probe, read_probe, NxgError
    c = copy_probe(1 << 24, 2)
    r = read_probe(1 << 24, 2)
    say("copy probe %.0f GB/s, read probe %.0f GB/s (16 MiB)" % (c, r))
    assert 10.0 < c < 20000.0 and 10.0 < r < 20000.0
    with pytest.raises(NxgError, match="EINVAL"):
        read_probe(1024, 1)
