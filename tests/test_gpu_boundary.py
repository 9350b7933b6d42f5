"""The boundary's failure and bookkeeping paths: allocator failures at every
allocation of a build and of a run (NXG_ENOMEM, no handle, nothing leaked),
the shuffled work-item schedule (results independent of the order in which
sub-shards are processed, Sec. II-A), torch.autograd.gradcheck of the
weighted-PageRank Function, device-side run statistics, and the bound on
captured runs kept by a handle."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import rmatgen
import paper_1510_06916_amd as nx
from paper_1510_06916_amd import DSSS, WeightedPageRank, _lib
from gpu_util import rel_l1, say, to_dev

pytestmark = pytest.mark.gpu


class FailingAllocator:
    """Forwards to torch's caching allocator, records the live pointers the
    library holds, and returns NULL at allocation number fail_at (0-based)."""

    def __init__(self, fail_at=None):
        self.fail_at = fail_at
        self.count = 0
        self.live = {}

        def _alloc(nbytes, stream, ctx):
            k = self.count
            self.count += 1
            if self.fail_at is not None and k == self.fail_at:
                return None
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                       int(stream or 0))
            except Exception:
                return None
            self.live[int(p)] = int(nbytes)
            return p

        def _free(ptr, nbytes, stream, ctx):
            self.live.pop(int(ptr), None)
            torch.cuda.caching_allocator_delete(int(ptr))

        self.refs = (_lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free))

    def __enter__(self):
        nx.install_torch_allocator()
        _lib.check(_lib.lib().nxg_set_allocator(self.refs[0], self.refs[1], None), "nxg_set_allocator")
        return self

    def __exit__(self, *exc):
        a, f = nx._alloc_refs
        _lib.check(_lib.lib().nxg_set_allocator(a, f, None), "nxg_set_allocator")


def _build_raw(src_d, dst_d, n, w_d, flags, order):
    d = _lib.BuildDesc(n=n, m=src_d.numel(), d_src=src_d.data_ptr(), d_dst=dst_d.data_ptr(),
                       d_weight=w_d.data_ptr() if w_d is not None else None, interval=256, tile=512,
                       chunk=256, value_bytes=8, flags=flags, order=order)
    h = ctypes.c_void_p(12345)
    rc = _lib.lib().nxg_dsss_build(ctypes.byref(d), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                   ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("flags,order,weighted", [
    (_lib.NXG_BUILD_RELABEL | _lib.NXG_BUILD_TRANSPOSE | _lib.NXG_BUILD_KEEP_PERM, _lib.NXG_ORDER_SRC, True),
    (_lib.NXG_BUILD_SYMMETRIZE | _lib.NXG_BUILD_DEGREE, _lib.NXG_ORDER_DST, False),
])
def test_enomem_at_every_build_allocation(gpu_device, flags, order, weighted):
    n = 3000
    src, dst = rmatgen.rmat_edges(12, 4, seed=71)
    src, dst = (src % n).astype(np.int32), (dst % n).astype(np.int32)
    src_d, dst_d = to_dev(src, gpu_device), to_dev(dst, gpu_device)
    w_d = torch.rand(len(src), device=gpu_device, dtype=torch.float32) if weighted else None
    torch.cuda.synchronize()
    with FailingAllocator() as probe:
        rc, h = _build_raw(src_d, dst_d, n, w_d, flags, order)
        assert rc == _lib.NXG_OK
        total = probe.count
        held = dict(probe.live)
        assert _lib.lib().nxg_dsss_destroy(h) == _lib.NXG_OK
        torch.cuda.synchronize()
        assert probe.live == {}
    say("build makes %d allocations and keeps %d" % (total, len(held)))
    assert total >= 5
    for k in range(total):
        with FailingAllocator(fail_at=k) as fa:
            rc, h = _build_raw(src_d, dst_d, n, w_d, flags, order)
            torch.cuda.synchronize()
            assert rc == _lib.NXG_ENOMEM, (k, rc, _lib.lib().nxg_last_error())
            assert h.value is None, "a handle was returned after a failed allocation"
            assert fa.live == {}, "allocation %d failed: %d buffers leaked" % (k, len(fa.live))
    # the library still works afterwards
    g = DSSS.build(src_d, dst_d, n, interval=256, tile=512, value_bytes=8)
    x, _ = g.pagerank(5, dtype=torch.float64)
    ref, _ = oracle.pagerank(n, src, dst, iters=5)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12


def test_enomem_at_every_run_allocation(gpu_device):
    n = 1 << 12
    src, dst = rmatgen.rmat_edges(12, 8, seed=72)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=512, tile=1024,
                   chunk=256, relabel=True, order="src")
    t = torch.rand(n, device=gpu_device, dtype=torch.float64)
    t /= t.sum()
    out = torch.empty(n, dtype=torch.float64, device=gpu_device)
    for prog_kw in (dict(teleport=t, tol=1e-9), dict(capture=True)):
        with FailingAllocator() as probe:
            g.pagerank(40, dtype=torch.float64, out=out, **prog_kw)
            torch.cuda.synchronize()
            total = probe.count
        say("run %s: %d allocations" % (sorted(prog_kw), total))
        for k in range(total):
            with FailingAllocator(fail_at=k) as fa:
                with pytest.raises(_lib.NxgError) as e:
                    g.pagerank(41, dtype=torch.float64, out=out, **prog_kw)  # 41: a new capture
                torch.cuda.synchronize()
                assert e.value.status == _lib.NXG_ENOMEM
                assert fa.live == {}, "run allocation %d failed: %d buffers leaked" % (k, len(fa.live))
    ref, _ = oracle.pagerank(n, src, dst, iters=12)
    x, _ = g.pagerank(12, dtype=torch.float64)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12


def test_enomem_at_every_scc_and_multi_root_bfs_allocation(gpu_device):
    # each failure on a fresh handle (the first successful run keeps its
    # workspace in the handle); after the refused run the handle is destroyed
    # and nothing allocated through the hook may remain
    n = 1 << 12
    src, dst = rmatgen.rmat_edges(12, 8, seed=74)
    s_d, d_d = to_dev(src, gpu_device), to_dev(dst, gpu_device)

    def fresh():
        return DSSS.build(s_d, d_d, n, interval=512, tile=1024, chunk=256, relabel=True, order="src",
                          transpose=True, value_bytes=8)
    runs = (("scc", lambda g: g.scc()), ("bfs_multi", lambda g: g.bfs_multi([0, 1, 2])))
    for name, run in runs:
        g = fresh()
        with FailingAllocator() as probe:
            run(g)
            torch.cuda.synchronize()
            total = probe.count
        g.close()
        say("%s run: %d allocations" % (name, total))
        assert total >= 3
        for k in range(total):
            g = fresh()
            with FailingAllocator(fail_at=k) as fa:
                with pytest.raises(_lib.NxgError) as e:
                    run(g)
                torch.cuda.synchronize()
                assert e.value.status == _lib.NXG_ENOMEM, (name, k)
                g.close()
                torch.cuda.synchronize()
                assert fa.live == {}, "%s allocation %d failed: %d buffers left" % (name, k, len(fa.live))
    g = fresh()
    assert np.array_equal(g.scc()[0].cpu().numpy(), oracle.scc(n, src, dst)[0])


@pytest.mark.parametrize("order,relabel", [("dst", False), ("src", True)])
def test_shuffled_schedule(gpu_device, order, relabel, monkeypatch):
    # pieces of 2 chunks split the heavy tiles, so pieces, finishing segments
    # and tiles all change places
    monkeypatch.setenv("NXG_PIECE_CHUNKS", "2")
    n = 1 << 15
    src, dst = rmatgen.rmat_edges(15, 16, seed=73)
    s_d, d_d = to_dev(src, gpu_device), to_dev(dst, gpu_device)
    kw = dict(interval=4096, tile=2048, chunk=256, order=order, relabel=relabel)
    res = {}
    for shuf in (False, True):
        gp = DSSS.build(s_d, d_d, n, value_bytes=8, shuffle_schedule=shuf, **kw)
        gb = DSSS.build(s_d, d_d, n, value_bytes=4, shuffle_schedule=shuf, **kw)
        gw = DSSS.build(s_d, d_d, n, value_bytes=4, symmetrize=True, shuffle_schedule=shuf, **kw)
        gs = DSSS.build(s_d, d_d, n, value_bytes=8, transpose=True, shuffle_schedule=shuf, **kw)
        x, _ = gp.pagerank(10, dtype=torch.float64)
        lev, stb = gb.bfs(int(src[0]))
        lab, stw = gw.wcc()
        scc, _ = gs.scc()
        mlev, _ = gs.bfs_multi([int(src[0]), int(src[1]), 5])
        res[shuf] = (x.cpu().numpy(), lev.cpu().numpy(), lab.cpu().numpy(), stb, stw, scc.cpu().numpy(),
                     mlev.cpu().numpy())
    (x0, l0, c0, b0, w0, s0, m0), (x1, l1, c1, b1, w1, s1, m1) = res[False], res[True]
    assert np.array_equal(s1, s0) and np.array_equal(m1, m0)
    assert np.array_equal(s1, oracle.scc(n, src, dst)[0])
    say("shuffled schedule %s: pagerank rel L1 %.2e" % (order, rel_l1(x1, x0)))
    assert rel_l1(x1, x0) <= 1e-14
    assert np.array_equal(l1, l0) and np.array_equal(c1, c0)
    assert b1["changed_rounds"] == b0["changed_rounds"] and b1["max_level"] == b0["max_level"]
    assert w1["changed_rounds"] == w0["changed_rounds"]
    ref, _ = oracle.pagerank(n, src, dst, iters=10)
    assert rel_l1(x1, ref) <= 1e-12
    rl, _, _ = oracle.bfs(n, src, dst, int(src[0]))
    assert np.array_equal(l1, rl)


def test_gradcheck_weighted_pagerank(gpu_device):
    # n <= 50, FP64 inputs; the library stores weights in FP32, so eps = 1e-3
    # keeps the FP32 rounding of w +- eps (~3e-8) at ~3e-5 of the difference
    n = 40
    rng = np.random.default_rng(74)
    key = np.unique(rng.integers(0, n, 130) * n + rng.integers(0, n, 130))
    src, dst = (key // n).astype(np.int32), (key % n).astype(np.int32)
    assert (np.bincount(src, minlength=n) == 0).any()  # dangling vertices present
    w = rmatgen.row_normalized_weights(src, n, seed=174)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n,
                   weights=torch.from_numpy(w), transpose=True, keep_perm=True, value_bytes=8)
    wt = torch.from_numpy(w.astype(np.float64)).to(gpu_device).requires_grad_(True)
    t = rng.random(n)
    tt = torch.from_numpy(t / t.sum()).to(gpu_device).requires_grad_(True)

    def f(w_, t_):
        return WeightedPageRank.apply(w_, t_, g, 0.85, 1e-14, 100000)

    assert torch.autograd.gradcheck(f, (wt, tt), eps=1e-3, atol=1e-7, rtol=1e-3)


def test_device_stats_and_capture(gpu_device):
    n = 1 << 13
    src, dst = rmatgen.rmat_edges(13, 8, seed=75)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=1024, value_bytes=8)
    iters = 9
    ref, res = oracle.pagerank(n, src, dst, iters=iters)
    deg = np.bincount(src, minlength=n)
    for capture in (False, True):
        st_d = torch.full((4 * iters,), float("nan"), dtype=torch.float64, device=gpu_device)
        out = torch.empty(n, dtype=torch.float64, device=gpu_device)
        for rep in range(2):
            st_d.fill_(float("nan"))
            x, st = g.pagerank(iters, dtype=torch.float64, out=out, capture=capture, stats_out=st_d)
            s = st_d.cpu().numpy().reshape(iters, 4)
            assert np.allclose(s[:, 1], res, rtol=1e-9, atol=1e-18)
            assert np.allclose(s[:, 2], 1.0, atol=1e-12)
            assert (s[:, 3] == 0).all()
            # entry 0 of iteration 0: dangling mass of x^0 = 1/n per dangling vertex
            assert abs(s[0, 0] - (deg == 0).sum() / n) <= 1e-15
            assert abs(st["residual"] - res[-1]) <= 1e-9 * res[-1]
            assert rel_l1(x.cpu().numpy(), ref) <= 1e-12
    with pytest.raises(_lib.NxgError):  # not written by other programs
        gb = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, interval=1024, value_bytes=8)
        bad = _lib.RunDesc(program=_lib.NXG_BFS, dtype=_lib.NXG_I32, batch=1, max_iters=5,
                           roots=ctypes.cast((ctypes.c_int32 * 1)(0), ctypes.c_void_p),
                           d_values=out.data_ptr(), d_stats=st_d.data_ptr())
        gb._run(bad)


def test_captured_runs_are_bounded(gpu_device):
    # every call with another output buffer records a new graph with its own
    # workspace; the handle keeps at most 8, so device memory stops growing
    n = 1 << 15
    src, dst = rmatgen.rmat_edges(15, 8, seed=76)
    g = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n)
    outs = [torch.empty(n, dtype=torch.float32, device=gpu_device) for _ in range(20)]
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    g.pagerank(5, out=outs[0], capture=True)
    torch.cuda.synchronize()
    one = torch.cuda.memory_allocated() - base
    assert one > 0
    for o in outs[1:]:
        g.pagerank(5, out=o, capture=True)
    torch.cuda.synchronize()
    grown = torch.cuda.memory_allocated() - base
    say("one capture: %d bytes; after 20: %d bytes" % (one, grown))
    assert grown <= 8 * one + (1 << 20)
    ref, _ = oracle.pagerank(n, src, dst, iters=5)
    for o in (outs[0], outs[-1]):  # the oldest graph was released and is recorded again
        x, _ = g.pagerank(5, out=o, capture=True)
        assert rel_l1(x.cpu().numpy(), ref) <= 1e-5


def test_non_finite_inputs_are_refused(gpu_device):
    # NaN and infinite weights and teleport entries are refused; negative ones
    # are accepted (the iteration is linear in both, and gradient checks
    # perturb them below zero)
    n = 1 << 10
    src, dst = rmatgen.rmat_edges(10, 4, seed=75)
    s_d, d_d = to_dev(src, gpu_device), to_dev(dst, gpu_device)
    m = len(src)
    w = torch.rand(m, device=gpu_device, dtype=torch.float32) + 0.1
    for bad in (float("nan"), float("inf"), -float("inf")):
        wb = w.clone()
        wb[m // 2] = bad
        with pytest.raises(_lib.NxgError) as e:
            DSSS.build(s_d, d_d, n, interval=256, weights=wb, keep_perm=True, value_bytes=8)
        assert e.value.status == _lib.NXG_EINVAL
    g = DSSS.build(s_d, d_d, n, interval=256, weights=w, keep_perm=True, value_bytes=8)
    x_ok, _ = g.pagerank(5, dtype=torch.float64, weighted=True)
    wb = w.clone()
    wb[3] = float("nan")
    with pytest.raises(_lib.NxgError) as e:
        g.set_weights(wb)
    assert e.value.status == _lib.NXG_EINVAL
    # the refused weights were not stored (the LDS sums' order varies between
    # runs, so the two agree to rounding)
    x_again, _ = g.pagerank(5, dtype=torch.float64, weighted=True)
    assert rel_l1(x_again.cpu().numpy(), x_ok.cpu().numpy()) <= 1e-13
    t = torch.full((n,), 1.0 / n, dtype=torch.float64, device=gpu_device)
    for bad in (float("nan"), float("inf")):
        tb = t.clone()
        tb[n - 1] = bad
        with pytest.raises(_lib.NxgError) as e:
            g.pagerank(5, dtype=torch.float64, teleport=tb)
        assert e.value.status == _lib.NXG_EINVAL
    # a teleport with a negative entry runs (and matches the oracle), also
    # through the relabeled ids
    tn = t.clone()
    tn[7] = -2.0 / n
    tn[8] = 3.0 / n
    gr = DSSS.build(s_d, d_d, n, interval=256, relabel=True, value_bytes=8)
    ref, _ = oracle.pagerank(n, src, dst, iters=5, t=tn.cpu().numpy())
    for gg in (g, gr):
        x, _ = gg.pagerank(5, dtype=torch.float64, teleport=tn)
        assert np.abs(x.cpu().numpy() - ref).sum() / np.abs(ref).sum() <= 1e-12
