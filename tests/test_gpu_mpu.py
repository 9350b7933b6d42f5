"""Mixed-phase update (Sec. III-B3, Alg. 7) with host memory as the slower tier
(NXG_RUN_MPU): only Q source intervals keep their values in device memory, the
others are staged from pinned host memory row by row, and sub-shards between
two non-resident intervals pass through shard hubs in host memory. Budgets
force Q = 0 (the DPU), intermediate Q and Q = P (the SPU); results are
compared with the FP64 oracle, and the host traffic with the schedule's
count."""
import numpy as np
import pytest
import torch

import oracle
import rmatgen
from paper_1510_06916_amd import DSSS
from gpu_util import rel_l1, say, to_dev

pytestmark = pytest.mark.gpu


def budget_for(q, I, vb):
    # Q resident intervals: two values and an 8-byte accumulator per vertex,
    # plus one staged interval
    return q * I * (2 * vb + 8) + I * vb


def expected_host_bytes(n, I, T, P, Q, vb, iters):
    R = min(Q * I, n)
    n_tiles = -(-n // T)
    Nt = n_tiles - min(n_tiles, (Q * I) // T)
    rd = (n - R) * vb + Nt * (P - Q) * T * 8 + (n - R) * vb
    wr = (P - Q) * Nt * T * 8 + (n - R) * vb
    return rd * iters, wr * iters


@pytest.mark.parametrize("dtype,order,Q", [
    (torch.float64, "dst", 0), (torch.float64, "dst", 4), (torch.float64, "src", 8),
    (torch.float64, "src", 16), (torch.float32, "dst", 5), (torch.float32, "src", 0)])
def test_mpu_scale16(gpu_device, dtype, order, Q, monkeypatch):
    # whole items (no pieces), so the host traffic is the schedule's count exactly
    monkeypatch.setenv("NXG_PIECE_CHUNKS", "1000000")
    n, I, T = 1 << 16, 4096, 4096
    P = n // I
    src, dst = rmatgen.rmat_edges(16, 16, seed=81)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=I, tile=T, chunk=256,
                   value_bytes=8, order=order)
    vb = 8 if dtype == torch.float64 else 4
    iters = 10
    x, st = g.pagerank(iters, dtype=dtype, mpu_budget=budget_for(Q, I, vb))
    ref, _ = oracle.pagerank(n, src, dst, iters=iters)
    e = rel_l1(x.cpu().numpy(), ref)
    say("mpu scale 16 %s %s Q=%d: rel L1 %.2e, host read %d write %d" % (
        dtype, order, st["resident_intervals"], e, st["host_read_bytes"], st["host_write_bytes"]))
    assert st["resident_intervals"] == Q
    assert e <= (1e-12 if dtype == torch.float64 else 1e-5)
    rd, wr = expected_host_bytes(n, I, T, P, Q, vb, iters)
    assert (st["host_read_bytes"], st["host_write_bytes"]) == (rd, wr)
    # the plain (all resident) run gives the same vector
    xp, _ = g.pagerank(iters, dtype=dtype)
    assert rel_l1(x.cpu().numpy(), xp.cpu().numpy()) <= (1e-13 if dtype == torch.float64 else 1e-6)


@pytest.mark.parametrize("order,Q", [("dst", 0), ("dst", 5), ("src", 9), ("dst", 16)])
def test_mpu_pieces(gpu_device, order, Q, monkeypatch):
    # pieces of 2 chunks: resident tiles take many atomic adds into their
    # accumulators, non-resident (tile, row) items spread over hub slots of
    # their own, and the heavy first tile is split everywhere
    monkeypatch.setenv("NXG_PIECE_CHUNKS", "2")
    n, I, T = 1 << 16, 4096, 4096
    P = n // I
    src, dst = rmatgen.rmat_edges(16, 16, seed=84)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=I, tile=T, chunk=256,
                   value_bytes=8, order=order)
    iters = 8
    x, st = g.pagerank(iters, dtype=torch.float64, mpu_budget=budget_for(Q, I, 8))
    ref, _ = oracle.pagerank(n, src, dst, iters=iters)
    e = rel_l1(x.cpu().numpy(), ref)
    say("mpu pieces %s Q=%d: rel L1 %.2e, host read %d write %d" % (
        order, st["resident_intervals"], e, st["host_read_bytes"], st["host_write_bytes"]))
    assert st["resident_intervals"] == Q and e <= 1e-12
    rd, wr = expected_host_bytes(n, I, T, P, Q, 8, iters)
    # a piece of a non-resident tile writes (and the update reads) one more hub slot
    assert st["host_read_bytes"] >= rd and st["host_write_bytes"] >= wr
    assert (st["host_read_bytes"] - rd) % (T * 8) == 0 and (st["host_read_bytes"] - rd) == (st["host_write_bytes"] - wr)
    if Q == P:
        assert st["host_read_bytes"] == 0 and st["host_write_bytes"] == 0
    x32, _ = g.pagerank(iters, dtype=torch.float32, mpu_budget=budget_for(Q, I, 4))
    assert rel_l1(x32.cpu().numpy(), ref) <= 1e-5


def test_mpu_weighted_ragged_teleport_tolerance_warm_start(gpu_device):
    # n not a multiple of the interval: the last interval (and tile) is short
    n, I, T = 50000, 4096, 2048
    src, dst = rmatgen.rmat_edges(16, 8, seed=82)
    src, dst = (src % n).astype(np.int32), (dst % n).astype(np.int32)
    key = np.unique(src.astype(np.int64) * n + dst)
    src, dst = (key // n).astype(np.int32), (key % n).astype(np.int32)
    w = rmatgen.row_normalized_weights(src, n, seed=182)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=I, tile=T, chunk=256,
                   value_bytes=8, weights=torch.from_numpy(w), keep_perm=True)
    rng = np.random.default_rng(3)
    t = rng.random(n)
    t /= t.sum()
    tt = torch.from_numpy(t).to(gpu_device)
    budget = budget_for(3, I, 8)
    ref, res = oracle.pagerank(n, src, dst, iters=400, w=w.astype(np.float64), t=t, tol=1e-11)
    x, st = g.pagerank(400, dtype=torch.float64, tol=1e-11, teleport=tt, weighted=True, mpu_budget=budget)
    say("mpu weighted tol: %d iterations (oracle %d), Q=%d" % (st["iterations"], len(res),
                                                                st["resident_intervals"]))
    assert st["converged"] == 1 and st["iterations"] == len(res) and st["resident_intervals"] == 3
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12
    # 6 iterations, then 4 more from that vector == 10 iterations
    r10, _ = oracle.pagerank(n, src, dst, iters=10, w=w.astype(np.float64), t=t)
    x6, _ = g.pagerank(6, dtype=torch.float64, teleport=tt, weighted=True, mpu_budget=budget)
    x10, _ = g.pagerank(4, dtype=torch.float64, teleport=tt, weighted=True, x0=x6, mpu_budget=budget)
    assert rel_l1(x10.cpu().numpy(), r10) <= 1e-12
    # zero iterations give x^0 = t
    x0, _ = g.pagerank(0, dtype=torch.float64, teleport=tt, weighted=True, mpu_budget=budget)
    assert np.array_equal(x0.cpu().numpy(), t)


def test_mpu_scale20_budget_from_environment(gpu_device, monkeypatch):
    n, I, T = 1 << 20, 65536, 16384
    src_d, dst_d = rmatgen.rmat_edges_gpu(20, 16, 83, device=gpu_device)
    src, dst = src_d.cpu().numpy(), dst_d.cpu().numpy()
    g = DSSS.build(src_d, dst_d, n, interval=I, tile=T, value_bytes=8)
    # a 5 MiB budget holds 4 of the 16 intervals of FP32 values (16 bytes per
    # resident vertex, one 256 KiB interval staged)
    monkeypatch.setenv("NXG_VERTEX_BUDGET_MB", "5")
    iters = 10
    x, st = g.pagerank(iters, dtype=torch.float32, mpu_budget=0)
    ref, _ = oracle.pagerank(n, src, dst, iters=iters)
    e = rel_l1(x.cpu().numpy(), ref)
    say("mpu scale 20: Q=%d of 16, rel L1 %.2e, %.1f ms, host read %.0f MB write %.0f MB" % (
        st["resident_intervals"], e, st["device_ms"], st["host_read_bytes"] / 1e6,
        st["host_write_bytes"] / 1e6))
    assert st["resident_intervals"] == 4
    assert e <= 1e-5
    x64, _ = g.pagerank(iters, dtype=torch.float64, mpu_budget=budget_for(2, I, 8))
    xp64, _ = g.pagerank(iters, dtype=torch.float64)
    e64, ep64 = rel_l1(x64.cpu().numpy(), ref), rel_l1(xp64.cpu().numpy(), ref)
    # FP64 sums of k positive terms taken in another order than the oracle's
    # differ by at most (k - 1) u relative; the L1 error of one iteration is
    # then at most u * (largest in-degree), and each of the 10 iterations adds
    # at most that much (the iteration contracts old errors by d < 1). At scale
    # 16 this is below 1e-12; here the hubs are larger
    kmax = int(np.bincount(dst, minlength=n).max())
    bound = iters * kmax * np.finfo(np.float64).eps / 2
    say("mpu scale 20 fp64: rel L1 %.2e (plain run %.2e), bound %.2e (max in-degree %d)" % (
        e64, ep64, bound, kmax))
    assert e64 <= bound and ep64 <= bound
    assert rel_l1(x64.cpu().numpy(), xp64.cpu().numpy()) <= bound


def test_mpu_refusals(gpu_device):
    n = 1 << 12
    src, dst = rmatgen.rmat_edges(12, 8, seed=84)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=1000, value_bytes=8)
    with pytest.raises(Exception, match="power of two"):
        g.pagerank(3, mpu_budget=1 << 20)
    gr = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=1024, relabel=True)
    with pytest.raises(Exception, match="natural vertex ids"):
        gr.pagerank(3, mpu_budget=1 << 20)
    g2 = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=1024, value_bytes=8)
    with pytest.raises(Exception, match="budget"):
        g2.pagerank(3, mpu_budget=0)
    with pytest.raises(Exception):
        g2.pagerank(3, mpu_budget=1 << 20, capture=True, out=torch.empty(n, device=gpu_device))
