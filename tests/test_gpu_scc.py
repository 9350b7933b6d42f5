"""Strongly connected components on the GPU against the oracle, bit-exact
(label = smallest caller id of the component)."""
import numpy as np
import pytest
import torch

import oracle
import rmatgen
from paper_1510_06916_amd import DSSS, _lib
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def _check(g, n, src, dst, what):
    say("scc " + what)
    ref, k = oracle.scc(n, src, dst)
    lab, st = g.scc()
    lab = lab.cpu().numpy()
    assert np.array_equal(lab, ref), what
    assert st["converged"] == 1 and st["iterations"] >= 1
    return st


@pytest.mark.parametrize("scale,ef,interval,tile,order,relabel", [
    (12, 4, 512, 0, "dst", False), (14, 8, 1000, 0, "dst", False), (14, 8, 2048, 4096, "src", False),
    (13, 16, 1024, 8192, "dst", True), (15, 8, 4096, 0, "src", True), (16, 16, 16384, 0, "dst", False)])
def test_scc_rmat_layouts(gpu_device, scale, ef, interval, tile, order, relabel):
    n = 1 << scale
    src, dst = rmatgen.rmat_edges(scale, ef, seed=scale + 7)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=interval, tile=tile,
                   order=order, relabel=relabel, transpose=True)
    st = _check(g, n, src, dst, "scale=%d ef=%d I=%d T=%d %s relabel=%s" % (scale, ef, interval, tile,
                                                                           order, relabel))
    # a second run on the same handle reuses its workspace
    lab2, st2 = g.scc()
    assert np.array_equal(lab2.cpu().numpy(), oracle.scc(n, src, dst)[0])
    assert st2["iterations"] == st["iterations"] and st2["changed_rounds"] == st["changed_rounds"]


def test_scc_split_tiles_ragged_n_degree(gpu_device, monkeypatch):
    # n not a multiple of any tile or interval, pieces of 2 chunks (split tiles
    # and hub slots), a hub every vertex points at and which points back at a
    # few, ids without edges dropped by degreeing
    n = 70001
    rs, rd = rmatgen.rmat_edges(16, 6, seed=23)
    rs, rd = rs % n, rd % n
    hub_in = np.arange(0, n, 3, dtype=np.int64)
    src = np.concatenate([rs, hub_in, np.full(50, 11)]).astype(np.int32)
    dst = np.concatenate([rd, np.full(len(hub_in), 11), np.arange(50) * 997 % n]).astype(np.int32)
    monkeypatch.setenv("NXG_PIECE_CHUNKS", "2")
    for order, relabel, degree in (("dst", False, False), ("src", True, True), ("dst", True, True)):
        g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=3000, tile=4096,
                       chunk=256, order=order, relabel=relabel, degree=degree, transpose=True)
        _check(g, n, src, dst, "hub n=%d %s relabel=%s degree=%s" % (n, order, relabel, degree))


def test_scc_small_graphs(gpu_device):
    rng = np.random.default_rng(31)
    for t in range(12):
        n = int(rng.integers(1, 300))
        m = int(rng.integers(1, 4 * n))
        src = rng.integers(0, n, m).astype(np.int32)
        dst = rng.integers(0, n, m).astype(np.int32)
        g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=min(64, n),
                       tile=64 if n >= 64 else 0,
                       order=("dst", "src")[t % 2], relabel=bool(t % 3 == 0), transpose=True)
        _check(g, n, src, dst, "random n=%d m=%d" % (n, m))


def test_scc_cycle_dag_and_chain(gpu_device):
    n = 2000
    v = np.arange(n, dtype=np.int32)
    # one long cycle written top down: the colour walks n - 1 passes
    g = DSSS.build(to_dev((v + 1) % n, gpu_device), to_dev(v, gpu_device), n, interval=256, transpose=True)
    st = _check(g, n, (v + 1) % n, v, "cycle")
    assert st["iterations"] == 1
    # two cycles and a chain of singletons hanging off them
    src = np.concatenate([v[:100], v[100:200], v[200:n - 1]]).astype(np.int32)
    dst = np.concatenate([(v[:100] + 1) % 100, 100 + (v[100:200] - 99) % 100, v[200:n - 1] + 1]).astype(np.int32)
    src = np.concatenate([src, [150, 5]]).astype(np.int32)
    dst = np.concatenate([dst, [200, 120]]).astype(np.int32)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=512, order="src",
                   transpose=True)
    _check(g, n, src, dst, "cycles and chain")
    # a DAG: every vertex is its own component
    a = np.random.default_rng(4).integers(0, n, (2, 8000))
    s2, d2 = np.minimum(a[0], a[1]), np.maximum(a[0], a[1])
    keep = s2 != d2
    s2, d2 = s2[keep].astype(np.int32), d2[keep].astype(np.int32)
    g = DSSS.build(to_dev(d2, gpu_device), to_dev(s2, gpu_device), n, interval=1024, transpose=True)
    _check(g, n, d2, s2, "dag")


def test_scc_empty_graph(gpu_device):
    e = torch.zeros(0, dtype=torch.int32, device=gpu_device)
    g = DSSS.build(e, e, 37, interval=16, transpose=True)
    lab, st = g.scc()
    assert np.array_equal(lab.cpu().numpy(), np.arange(37))


def test_scc_refusals_and_pass_budget(gpu_device):
    n = 1 << 12
    src, dst = rmatgen.rmat_edges(12, 4, seed=3)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=512)
    with pytest.raises(_lib.NxgError) as e:
        g.scc()
    assert e.value.status == _lib.NXG_EINVAL  # no reversed layout
    gt = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=512, transpose=True)
    lab, st = gt.scc(max_passes=1)
    assert st["status"] == _lib.NXG_ENOTCONV and st["converged"] == 0
    lab, st = gt.scc()
    assert np.array_equal(lab.cpu().numpy(), oracle.scc(n, src, dst)[0])
