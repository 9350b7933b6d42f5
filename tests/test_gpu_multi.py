"""Many graphs per launch against plain per-graph GPU runs and the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import rmatgen
from paper_1510_06916_amd import DSSS, MultiDSSS, NxgError
from gpu_util import rel_l1, say, to_dev

pytestmark = pytest.mark.gpu

PERSISTENT_OFF = ("the single persistent launch (workgroups waiting on per-graph iteration "
                  "counters) did not finish on MI355X; it is switched off and its cause is "
                  "not known")


def _graphs(count, device):
    rng = np.random.default_rng(77)
    out = []
    for g in range(count):
        scale = int(rng.integers(6, 14))
        ef = int(rng.integers(4, 17))
        src, dst = rmatgen.rmat_edges(scale, ef, seed=4000 + g)
        out.append((src, dst, 1 << scale))
    return out


def test_multi_batch_matches_plain_and_oracle(gpu_device):
    gs = _graphs(24, gpu_device)
    say("multi: %d graphs, %d edges" % (len(gs), sum(len(s) for s, _, _ in gs)))
    mg = MultiDSSS.build([(to_dev(s, gpu_device), to_dev(d, gpu_device), n) for s, d, n in gs],
                         tile=1024)
    xs, st = mg.pagerank(30)
    assert st["iterations"] == 30
    for i, (s, d, n) in enumerate(gs):
        ref, _ = oracle.pagerank(n, s, d, iters=30)
        assert rel_l1(xs[i].cpu().numpy(), ref) <= 1e-5, i
        if i % 6 == 0:
            g = DSSS.build(to_dev(s, gpu_device), to_dev(d, gpu_device), n, tile=1024)
            xp, _ = g.pagerank(30, dtype=torch.float32)
            assert rel_l1(xs[i].cpu().numpy(), xp.cpu().numpy()) <= 1e-6


@pytest.mark.parametrize("order,relabel", [("src", False), ("src", True)])
def test_multi_source_order_and_relabel(gpu_device, order, relabel):
    gs = _graphs(12, gpu_device)
    say("multi: order=%s relabel=%s" % (order, relabel))
    mg = MultiDSSS.build([(to_dev(s, gpu_device), to_dev(d, gpu_device), n) for s, d, n in gs],
                         order=order, relabel=relabel)
    xs, st = mg.pagerank(25)
    assert st["iterations"] == 25
    for i, (s, d, n) in enumerate(gs):
        ref, _ = oracle.pagerank(n, s, d, iters=25)
        assert rel_l1(xs[i].cpu().numpy(), ref) <= 1e-5, i
    # caller-owned outputs, and the handle's workspaces reused by a second run
    outs = [torch.full((n,), -1.0, dtype=torch.float32, device=gpu_device) for _, _, n in gs]
    xo, _ = mg.pagerank(25, out=outs)
    for i in range(len(gs)):
        assert xo[i].data_ptr() == outs[i].data_ptr()
        assert rel_l1(outs[i].cpu().numpy(), xs[i].cpu().numpy()) <= 1e-7, i
    with pytest.raises(ValueError):
        mg.pagerank(3, out=outs[:-1])


@pytest.mark.parametrize("relabel", [False, True])
def test_multi_capture_replays(gpu_device, relabel):
    # the recorded run replays into new output buffers each time, matches the
    # eager run, and is recorded again when the damping changes
    gs = _graphs(10, gpu_device)
    mg = MultiDSSS.build([(to_dev(s, gpu_device), to_dev(d, gpu_device), n) for s, d, n in gs],
                         order="src", relabel=relabel)
    xe, _ = mg.pagerank(20)
    xe = [x.clone() for x in xe]
    for rep in range(3):
        damping = 0.85 if rep < 2 else 0.7
        say("multi capture relabel=%d replay %d damping %.2f" % (relabel, rep, damping))
        outs = [torch.full((n,), -1.0, dtype=torch.float32, device=gpu_device) for _, _, n in gs]
        xc, st = mg.pagerank(20, damping=damping, out=outs, capture=True)
        torch.cuda.synchronize()
        assert st["iterations"] == 20
        for i, (s, d, n) in enumerate(gs):
            if damping == 0.85:
                assert rel_l1(xc[i].cpu().numpy(), xe[i].cpu().numpy()) <= 1e-6, i
            elif i % 3 == 0:
                ref, _ = oracle.pagerank(n, s, d, iters=20, d=0.7)
                assert rel_l1(xc[i].cpu().numpy(), ref) <= 1e-5, i


def test_multi_persistent_flag_is_refused(gpu_device):
    gs = _graphs(2, gpu_device)
    mg = MultiDSSS.build([(to_dev(s, gpu_device), to_dev(d, gpu_device), n) for s, d, n in gs])
    with pytest.raises(NxgError, match="EUNSUPPORTED"):
        mg.pagerank(3, persistent=True)


@pytest.mark.skip(reason=PERSISTENT_OFF)
def test_multi_persistent_matches_plain_and_oracle(gpu_device):
    gs = _graphs(24, gpu_device)
    mg = MultiDSSS.build([(to_dev(s, gpu_device), to_dev(d, gpu_device), n) for s, d, n in gs],
                         tile=1024)
    xs, _ = mg.pagerank(30, persistent=True)
    for i, (s, d, n) in enumerate(gs):
        ref, _ = oracle.pagerank(n, s, d, iters=30)
        assert rel_l1(xs[i].cpu().numpy(), ref) <= 1e-5, i


@pytest.mark.skip(reason=PERSISTENT_OFF)
def test_multi_persistent_wait_limit_reports_error(gpu_device, monkeypatch):
    gs = _graphs(8, gpu_device)
    mg = MultiDSSS.build([(to_dev(s, gpu_device), to_dev(d, gpu_device), n) for s, d, n in gs],
                         tile=256)
    monkeypatch.setenv("NXG_SPIN_LIMIT", "0")
    with pytest.raises(NxgError, match="EDEVICE"):
        mg.pagerank(30, persistent=True)
