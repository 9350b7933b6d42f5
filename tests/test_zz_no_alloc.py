"""PageRank through the allocation-free entry point (nxg_run_noalloc) against the
allocating one (nxg_run) and the FP64 oracle, on two calls in a row (the second
on a smaller graph), with an allocator hook that counts every device allocation
the library asks for during the calls."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import rmatgen
import paper_1510_06916_amd as nx
from paper_1510_06916_amd import DSSS, _lib
from gpu_util import rel_l1, say, to_dev

pytestmark = pytest.mark.gpu


class CountingAllocator:
    """Forwards to torch's caching allocator and counts the calls."""

    def __init__(self):
        self.allocs = 0
        self.frees = 0

        def _alloc(nbytes, stream, ctx):
            self.allocs += 1
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                          int(stream or 0))
            except Exception:
                return None

        def _free(ptr, nbytes, stream, ctx):
            self.frees += 1
            torch.cuda.caching_allocator_delete(int(ptr))

        self.refs = (_lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free))

    def __enter__(self):
        nx.install_torch_allocator()
        _lib.check(_lib.lib().nxg_set_allocator(self.refs[0], self.refs[1], None), "nxg_set_allocator")
        return self

    def __exit__(self, *exc):
        a, f = nx._alloc_refs
        _lib.check(_lib.lib().nxg_set_allocator(a, f, None), "nxg_set_allocator")


def graph(scale, ef, seed, dev, **kw):
    src, dst = rmatgen.rmat_edges(scale, ef, seed=seed)
    n = 1 << scale
    g = DSSS.build(to_dev(src, dev), to_dev(dst, dev), n, **kw)
    return g, src, dst, n


@pytest.mark.parametrize("dtype,kw", [
    (torch.float64, dict(P=4, value_bytes=8)),
    (torch.float32, dict(interval=2048, tile=4096, chunk=512, order="src", relabel=True)),
])
def test_noalloc_matches_nxg_run_two_calls(gpu_device, dtype, kw):
    bar_run = 1e-12 if dtype == torch.float64 else 1e-6
    bar_orc = 1e-12 if dtype == torch.float64 else 1e-5
    big = graph(15, 16, 11, gpu_device, **kw)
    small = graph(11, 8, 12, gpu_device, **kw)
    with CountingAllocator() as ca:
        for name, (g, src, dst, n) in (("scale 15", big), ("scale 11", small)):
            iters = 12
            say("noalloc %s dtype=%s n=%d m=%d" % (name, dtype, n, len(src)))
            ref, _ = oracle.pagerank(n, src, dst, iters=iters)
            x_run, st_run = g.pagerank(iters, dtype=dtype)
            out = torch.full((n,), float("nan"), dtype=dtype, device=gpu_device)
            torch.cuda.synchronize()
            a0, f0 = ca.allocs, ca.frees
            x, st = g.pagerank_noalloc(iters, out)
            torch.cuda.synchronize()
            assert (ca.allocs, ca.frees) == (a0, f0), "nxg_run_noalloc went through the allocator"
            xh = x.cpu().numpy()
            assert np.isfinite(xh).all()
            assert rel_l1(xh, x_run.cpu().numpy()) <= bar_run
            assert rel_l1(xh, ref) <= bar_orc
            assert st["iterations"] == iters and st_run["iterations"] == iters
            assert abs(st["residual"] - st_run["residual"]) <= 1e-6 * max(st_run["residual"], 1e-30)


def test_noalloc_tolerance_teleport_weighted(gpu_device):
    # FP64: a tolerance stop with a teleport vector, then a weighted run, each twice
    g, src, dst, n = graph(12, 8, 13, gpu_device, P=2, value_bytes=8, keep_perm=True)
    rng = np.random.default_rng(5)
    t = rng.random(n)
    t /= t.sum()
    tt = torch.from_numpy(t).to(gpu_device)
    ref, res = oracle.pagerank(n, src, dst, iters=500, t=t, tol=1e-10)
    for rep in range(2):
        out = torch.empty(n, dtype=torch.float64, device=gpu_device)
        x, st = g.pagerank_noalloc(500, out, tol=1e-10, teleport=tt)
        say("noalloc tol run %d: iterations %d (oracle %d)" % (rep, st["iterations"], len(res)))
        assert st["converged"] == 1 and st["iterations"] == len(res)
        assert rel_l1(x.cpu().numpy(), ref) <= 1e-12
    w = rmatgen.uniform_f32(105, len(src), lo=0.1, hi=1.0)
    gw = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), n, P=2, value_bytes=8,
                    weights=torch.from_numpy(np.asarray(w, dtype=np.float32)).to(gpu_device),
                    keep_perm=True)
    refw, _ = oracle.pagerank(n, src, dst, iters=9, w=np.asarray(w, dtype=np.float64))
    for rep in range(2):
        out = torch.empty(n, dtype=torch.float64, device=gpu_device)
        x, _ = gw.pagerank_noalloc(9, out, weighted=True)
        assert rel_l1(x.cpu().numpy(), refw) <= 1e-12


def test_noalloc_refusals(gpu_device):
    g, src, dst, n = graph(10, 8, 14, gpu_device, P=2, value_bytes=8)
    cap = _lib.lib().nxg_noalloc_scratch_bytes()
    assert cap == 64 << 20
    out = torch.empty(n, dtype=torch.float64, device=gpu_device)
    # statistics of 32 bytes per iteration: 3M iterations need more than the array
    with pytest.raises(_lib.NxgError, match="scratch region holds"):
        g.pagerank_noalloc(3_000_000, out, tol=1e-300)
    # a piece size no earlier run has planned
    d = _lib.RunDesc(program=_lib.NXG_PAGERANK, dtype=_lib.NXG_F64, batch=1, damping=0.85,
                     max_iters=3, tol=0.0, d_values=out.data_ptr(), flags=0, piece_chunks=7)
    st = _lib.RunStats()
    rc = _lib.lib().nxg_run_noalloc(g._h, ctypes.byref(d), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                    ctypes.byref(st))
    assert rc == _lib.NXG_EINVAL and b"plan" in _lib.lib().nxg_last_error()
    d.piece_chunks = 0
    d.flags = _lib.NXG_RUN_CAPTURE
    rc = _lib.lib().nxg_run_noalloc(g._h, ctypes.byref(d), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                    ctypes.byref(st))
    assert rc == _lib.NXG_EINVAL
    # the handle still runs afterwards
    x, st = g.pagerank_noalloc(3, out)
    ref, _ = oracle.pagerank(n, src, dst, iters=3)
    assert rel_l1(x.cpu().numpy(), ref) <= 1e-12
