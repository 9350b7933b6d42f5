"""MI355X DSSS graph-iteration library: Python binding of include/nxgraph.h.

Every step of the graph method runs in the HIP library (libnxgraph.so); this
module only marshals torch tensors (device memory, streams) into the C ABI. It
raises if the library is not built or no GPU is visible -- there is no CPU path.

    g = DSSS.build(src, dst, n, P=32)          # int32 device tensors
    x, st = g.pagerank(iters=20, dtype=torch.float32)
    lev, st = g.bfs(root)
"""
import ctypes

import torch

from . import _lib
from ._lib import NxgError  # noqa: F401

__all__ = ["DSSS", "MultiDSSS", "NxgError", "WeightedPageRank", "abi_version",
           "install_torch_allocator", "tune", "copy_probe", "read_probe"]

_alloc_refs = None


def abi_version():
    return _lib.lib().nxg_abi_version()


def install_torch_allocator():
    """Routes every device allocation of the library through torch's caching
    allocator, so all device memory is torch's (idempotent)."""
    global _alloc_refs
    if _alloc_refs is not None:
        return

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                      int(stream or 0))
        except Exception:  # reported to the caller as NXG_ENOMEM
            return None

    def _free(ptr, nbytes, stream, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    refs = (_lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free))
    _lib.check(_lib.lib().nxg_set_allocator(refs[0], refs[1], None), "nxg_set_allocator")
    _alloc_refs = refs


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_i32(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA tensor" % name)
    if t.dtype != torch.int32:
        raise ValueError("%s must be int32" % name)
    return t.contiguous()


_DT = {torch.float32: _lib.NXG_F32, torch.float64: _lib.NXG_F64}


def copy_probe(nbytes=1 << 30, reps=10):
    """Attainable HBM bandwidth (read + write GB/s) of a plain streaming copy."""
    install_torch_allocator()
    g = ctypes.c_double(0.0)
    _lib.check(_lib.lib().nxg_copy_probe(int(nbytes), int(reps), _stream_handle(), ctypes.byref(g)),
               "nxg_copy_probe")
    return g.value


def read_probe(nbytes=1 << 30, reps=10):
    """Attainable HBM read bandwidth (GB/s) of a plain read-only stream."""
    install_torch_allocator()
    g = ctypes.c_double(0.0)
    _lib.check(_lib.lib().nxg_read_probe(int(nbytes), int(reps), _stream_handle(), ctypes.byref(g)),
               "nxg_read_probe")
    return g.value


def tune(src, dst, n, dtype=torch.float32, weights=None, batch=1, stream=None):
    """Times candidate layouts for PageRank on this graph; returns a dict with
    interval, tile, chunk, order (0 dst, 1 src), relabel, pairs, piece_chunks,
    ms_per_iter, candidates and width. batch > 1 tunes batched personalised
    PageRank (FP32): width is then the columns per pass (build with
    value_bytes=8*width) and ms_per_iter covers the whole batch."""
    install_torch_allocator()
    src = _dev_i32(src, "src")
    dst = _dev_i32(dst, "dst")
    w = None if weights is None else weights.to(device=src.device, dtype=torch.float32).contiguous()
    d = _lib.BuildDesc(n=int(n), m=src.numel(), d_src=src.data_ptr() if src.numel() else None,
                       d_dst=dst.data_ptr() if dst.numel() else None,
                       d_weight=w.data_ptr() if w is not None else None, interval=0, tile=0,
                       chunk=0, value_bytes=8, flags=0, order=0)
    r = _lib.TuneResult()
    prog = _lib.NXG_PAGERANK_WEIGHTED if w is not None else _lib.NXG_PAGERANK
    with torch.cuda.device(src.device):
        _lib.check(_lib.lib().nxg_tune(ctypes.byref(d), prog, _DT[dtype], int(batch),
                                       _stream_handle(stream), ctypes.byref(r)), "nxg_tune")
    return {k: getattr(r, k) for k, _ in r._fields_}


class DSSS:
    """A graph stored as destination-sorted sub-shards on one GPU."""

    def __init__(self, handle, device):
        self._h = handle
        self.device = device
        self._info = None
        self.weights_version = 0

    # ---- construction ---------------------------------------------------
    @classmethod
    def build(cls, src, dst, n, P=None, interval=None, weights=None, tile=0, chunk=0,
              value_bytes=0, keep_perm=False, transpose=False, symmetrize=False, dedup=False,
              order="dst", relabel=False, scatter=False, degree=False, host_stream=False,
              pairs=False, shuffle_schedule=False, stream=None):
        """scatter=True builds the coarse-grained source-sorted layout
        (NXG_BUILD_SCATTER) that only pagerank(..., scatter=True) runs.
        degree=True drops the ids that appear in no edge (NXG_BUILD_DEGREE);
        vectors stay indexed by the caller's n ids. host_stream=True keeps the
        edge stream in pinned host memory and streams it every iteration
        (NXG_BUILD_HOST_STREAM; PageRank only). pairs=True (with order="src")
        packs two destinations of one source per word (NXG_BUILD_PAIRS; plain
        PageRank only). shuffle_schedule=True issues the work items in a seeded
        random order (NXG_BUILD_SHUFFLE_SCHEDULE, a debug check of order freedom)."""
        install_torch_allocator()
        src = _dev_i32(src, "src")
        dst = _dev_i32(dst, "dst")
        if src.numel() != dst.numel():
            raise ValueError("src and dst differ in length")
        n = int(n)
        if interval is None:
            interval = 0 if P is None else -(-n // int(P))
        w = None
        if weights is not None:
            w = weights.to(device=src.device, dtype=torch.float32).contiguous()
            if w.numel() != src.numel():
                raise ValueError("weights must have one entry per edge")
        flags = ((_lib.NXG_BUILD_KEEP_PERM if keep_perm else 0) |
                 (_lib.NXG_BUILD_TRANSPOSE if transpose else 0) |
                 (_lib.NXG_BUILD_SYMMETRIZE if symmetrize else 0) |
                 (_lib.NXG_BUILD_DEDUP if dedup else 0) |
                 (_lib.NXG_BUILD_RELABEL if relabel else 0) |
                 (_lib.NXG_BUILD_SCATTER if scatter else 0) |
                 (_lib.NXG_BUILD_DEGREE if degree else 0) |
                 (_lib.NXG_BUILD_HOST_STREAM if host_stream else 0) |
                 (_lib.NXG_BUILD_PAIRS if pairs else 0) |
                 (_lib.NXG_BUILD_SHUFFLE_SCHEDULE if shuffle_schedule else 0))
        d = _lib.BuildDesc(n=n, m=src.numel(), d_src=src.data_ptr() if src.numel() else None,
                           d_dst=dst.data_ptr() if dst.numel() else None,
                           d_weight=w.data_ptr() if w is not None else None,
                           interval=int(interval), tile=int(tile), chunk=int(chunk),
                           value_bytes=int(value_bytes), flags=flags,
                           order={"dst": _lib.NXG_ORDER_DST, "src": _lib.NXG_ORDER_SRC}[order])
        h = ctypes.c_void_p()
        with torch.cuda.device(src.device):
            _lib.check(_lib.lib().nxg_dsss_build(ctypes.byref(d), _stream_handle(stream),
                                                 ctypes.byref(h)), "nxg_dsss_build")
        return cls(h, src.device)

    def close(self):
        if self._h:
            _lib.lib().nxg_dsss_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        if self._info is None:
            inf = _lib.DsssInfo()
            _lib.check(_lib.lib().nxg_dsss_info_get(self._h, ctypes.byref(inf)), "nxg_dsss_info_get")
            self._info = {k: getattr(inf, k) for k, _ in inf._fields_}
        return self._info

    @property
    def n(self):
        return self.info()["n"]

    @property
    def m(self):
        return self.info()["m"]

    def vertex_map(self):
        """Caller id of every internal vertex (relabeled or degreed builds):
        int32 [n_kept]."""
        out = torch.empty(self.info()["n_kept"], dtype=torch.int32, device=self.device)
        _lib.check(_lib.lib().nxg_dsss_vertex_map(self._h, out.data_ptr(), _stream_handle()),
                   "nxg_dsss_vertex_map")
        return out

    def export(self, transposed=False, perm=False):
        """Offsets [P*P+1] (paper order j*P+i) and the stored edges in stream order."""
        inf = self.info()
        P, m = inf["P"], inf["m"]
        dev = self.device
        off = torch.empty(P * P + 1, dtype=torch.int64, device=dev)
        s = torch.empty(m, dtype=torch.int32, device=dev)
        t = torch.empty(m, dtype=torch.int32, device=dev)
        pm = torch.empty(m, dtype=torch.int32, device=dev) if perm else None
        _lib.check(_lib.lib().nxg_dsss_export(
            self._h, 1 if transposed else 0, off.data_ptr(), s.data_ptr() if m else None,
            t.data_ptr() if m else None, pm.data_ptr() if (pm is not None and m) else None,
            _stream_handle()), "nxg_dsss_export")
        out = {"offsets": off, "src": s, "dst": t}
        if perm:
            out["perm"] = pm
        return out

    # ---- programs -------------------------------------------------------
    def _run(self, desc, allow=()):
        st = _lib.RunStats()
        with torch.cuda.device(self.device):
            rc = _lib.check(_lib.lib().nxg_run(self._h, ctypes.byref(desc), _stream_handle(),
                                               ctypes.byref(st)), "nxg_run", allow=allow)
        out = st.as_dict()
        out["status"] = rc
        return out

    def pagerank(self, iters, damping=0.85, dtype=torch.float32, tol=0.0, teleport=None,
                 x0=None, weighted=False, out=None, capture=False, piece_chunks=0, scatter=False,
                 stats_out=None, mpu_budget=None):
        """stats_out: optional FP64 device tensor of 4 * iters entries that the run
        (and every replay of a captured one) fills with the per-iteration
        statistics (dangling mass, residual, sum of x, 0) without a host sync.
        capture=True records the run into a hipGraph kept by the handle (at most
        8 per handle, least recently used released first), replayed when a
        later call passes the same buffers. mpu_budget (bytes, or 0 for the
        environment variable NXG_VERTEX_BUDGET_MB) runs the mixed-phase update
        (NXG_RUN_MPU): only the vertex values that fit the budget stay in device
        memory, the rest in pinned host memory."""
        n = self.n
        if dtype not in _DT:
            raise ValueError("dtype must be float32 or float64")
        x = out if out is not None else torch.empty(n, dtype=dtype, device=self.device)
        flags = 0
        if x0 is not None:
            x.copy_(x0)
            flags |= _lib.NXG_RUN_WARM_START
        tp = None
        if teleport is not None:
            tp = teleport.to(device=self.device, dtype=dtype).contiguous()
        if scatter:
            flags |= _lib.NXG_RUN_SCATTER
        if mpu_budget is not None:
            flags |= _lib.NXG_RUN_MPU
        if capture:
            # a recorded graph reads and writes the buffers at the addresses it was
            # recorded with; it is only replayed for a call passing those addresses
            flags |= _lib.NXG_RUN_CAPTURE
        if stats_out is not None and (stats_out.dtype != torch.float64 or not stats_out.is_contiguous()
                                      or stats_out.numel() < 4 * int(iters)
                                      or stats_out.device != self.device):
            raise ValueError("stats_out must be a contiguous FP64 device tensor of 4 * iters entries")
        d = _lib.RunDesc(program=_lib.NXG_PAGERANK_WEIGHTED if weighted else _lib.NXG_PAGERANK,
                         dtype=_DT[dtype], batch=1, damping=float(damping),
                         max_iters=int(iters), tol=float(tol),
                         d_teleport=tp.data_ptr() if tp is not None else None, roots=None,
                         d_values=x.data_ptr(), flags=flags, piece_chunks=int(piece_chunks),
                         d_stats=stats_out.data_ptr() if stats_out is not None else None,
                         vertex_budget=int(mpu_budget or 0))
        st = self._run(d, allow=(_lib.NXG_ENOTCONV,))
        return x, st

    def pagerank_noalloc(self, iters, out, damping=0.85, tol=0.0, teleport=None, x0=None,
                         weighted=False):
        """PageRank through nxg_run_noalloc: the library allocates nothing during
        the call (its workspace is a per-device scratch array). out (FP32 or FP64,
        [n], on this device) receives x and fixes the dtype; teleport, if given,
        must already be a contiguous tensor of that dtype on this device."""
        if out.dtype not in _DT or not out.is_contiguous() or out.device != self.device:
            raise ValueError("out must be a contiguous FP32/FP64 tensor on the graph's device")
        flags = 0
        if x0 is not None:
            out.copy_(x0)
            flags |= _lib.NXG_RUN_WARM_START
        if teleport is not None and (teleport.dtype != out.dtype or not teleport.is_contiguous()
                                     or teleport.device != self.device):
            raise ValueError("teleport must be a contiguous tensor of out's dtype on the device")
        d = _lib.RunDesc(program=_lib.NXG_PAGERANK_WEIGHTED if weighted else _lib.NXG_PAGERANK,
                         dtype=_DT[out.dtype], batch=1, damping=float(damping),
                         max_iters=int(iters), tol=float(tol),
                         d_teleport=teleport.data_ptr() if teleport is not None else None,
                         roots=None, d_values=out.data_ptr(), flags=flags)
        st = _lib.RunStats()
        with torch.cuda.device(self.device):
            rc = _lib.check(_lib.lib().nxg_run_noalloc(self._h, ctypes.byref(d), _stream_handle(),
                                                       ctypes.byref(st)), "nxg_run_noalloc",
                            allow=(_lib.NXG_ENOTCONV,))
        res = st.as_dict()
        res["status"] = rc
        return out, res

    def ppr(self, seeds, iters, damping=0.85, tol=0.0, out=None, capture=False):
        """Batched personalised PageRank: column b teleports to seeds[b]; returns
        x [n, B] FP32 (B = len(seeds) <= 64). The graph must be built with
        value_bytes >= 8 * B. capture=True records the run into a hipGraph kept
        by the handle and replays it when a later call passes the same seed
        tensor (a device int32 tensor, whose contents may change) and out."""
        # a contiguous device int32 tensor is used in place (its pointer is kept)
        seeds = torch.as_tensor(seeds, dtype=torch.int32).to(self.device).contiguous()
        B = seeds.numel()
        x = out if out is not None else torch.empty((self.n, B), dtype=torch.float32,
                                                    device=self.device)
        flags = 0
        if capture:
            flags |= _lib.NXG_RUN_CAPTURE
        d = _lib.RunDesc(program=_lib.NXG_PAGERANK, dtype=_lib.NXG_F32, batch=B,
                         damping=float(damping), max_iters=int(iters), tol=float(tol),
                         d_teleport=None, roots=None, d_values=x.data_ptr(), flags=flags,
                         d_seeds=seeds.data_ptr())
        st = self._run(d, allow=(_lib.NXG_ENOTCONV,))
        return x, st

    def bfs(self, root, max_rounds=None):
        n = self.n
        lev = torch.empty(n, dtype=torch.int32, device=self.device)
        roots = (ctypes.c_int32 * 1)(int(root))
        d = _lib.RunDesc(program=_lib.NXG_BFS, dtype=_lib.NXG_I32, batch=1, damping=0.0,
                         max_iters=int(max_rounds if max_rounds is not None else n + 1), tol=0.0,
                         d_teleport=None, roots=ctypes.cast(roots, ctypes.c_void_p),
                         d_values=lev.data_ptr(), flags=0)
        return lev, self._run(d)

    def bfs_multi(self, roots, max_rounds=None):
        """BFS from 2..64 roots at once: levels [n, B] int32 (column b from
        roots[b]). The build needs value_bytes=8."""
        roots = [int(r) for r in roots]
        B = len(roots)
        lev = torch.empty((self.n, B), dtype=torch.int32, device=self.device)
        rr = (ctypes.c_int32 * B)(*roots)
        d = _lib.RunDesc(program=_lib.NXG_BFS, dtype=_lib.NXG_I32, batch=B, damping=0.0,
                         max_iters=int(max_rounds if max_rounds is not None else self.n + 1), tol=0.0,
                         d_teleport=None, roots=ctypes.cast(rr, ctypes.c_void_p),
                         d_values=lev.data_ptr(), flags=0)
        return lev, self._run(d, allow=(_lib.NXG_ENOTCONV,))

    def wcc(self, max_rounds=None):
        n = self.n
        lab = torch.empty(n, dtype=torch.int32, device=self.device)
        d = _lib.RunDesc(program=_lib.NXG_WCC, dtype=_lib.NXG_I32, batch=1, damping=0.0,
                         max_iters=int(max_rounds if max_rounds is not None else n + 1), tol=0.0,
                         d_teleport=None, roots=None, d_values=lab.data_ptr(), flags=0)
        return lab, self._run(d)

    def scc(self, max_passes=None):
        """Strongly connected components: label[v] = smallest caller id of v's
        component. Needs a build with transpose=True."""
        n = self.n
        lab = torch.empty(n, dtype=torch.int32, device=self.device)
        d = _lib.RunDesc(program=_lib.NXG_SCC, dtype=_lib.NXG_I32, batch=1, damping=0.0,
                         max_iters=int(max_passes if max_passes is not None else 2**31 - 1), tol=0.0,
                         d_teleport=None, roots=None, d_values=lab.data_ptr(), flags=0)
        return lab, self._run(d, allow=(_lib.NXG_ENOTCONV,))

    # ---- weighted PageRank and its adjoint ------------------------------
    def set_weights(self, w):
        """Replaces the stored edge weights (input edge order)."""
        w = w.detach().to(device=self.device, dtype=torch.float32).contiguous()
        if w.numel() != self.info()["m"]:
            raise ValueError("one weight per stored edge expected")
        with torch.cuda.device(self.device):
            _lib.check(_lib.lib().nxg_dsss_set_weights(self._h, w.data_ptr(), _stream_handle()),
                       "nxg_dsss_set_weights")
        self.weights_version += 1

    def pagerank_adjoint(self, xstar, gx, damping=0.85, tol=1e-12, max_iters=100000):
        """Returns (lambda, dL/dw [m] FP32 input edge order, dL/dt [n] FP64, stats)."""
        n, m = self.n, self.m
        xs = xstar.detach().to(device=self.device, dtype=torch.float64).contiguous()
        g = gx.detach().to(device=self.device, dtype=torch.float64).contiguous()
        lam = torch.empty(n, dtype=torch.float64, device=self.device)
        gw = torch.empty(m, dtype=torch.float32, device=self.device)
        gt = torch.empty(n, dtype=torch.float64, device=self.device)
        d = _lib.AdjointDesc(damping=float(damping), tol=float(tol), max_iters=int(max_iters),
                             d_xstar=xs.data_ptr(), d_gx=g.data_ptr(), d_lambda=lam.data_ptr(),
                             d_gw=gw.data_ptr() if m else None, d_gt=gt.data_ptr())
        st = _lib.RunStats()
        with torch.cuda.device(self.device):
            rc = _lib.check(_lib.lib().nxg_pagerank_adjoint(self._h, ctypes.byref(d),
                                                            _stream_handle(), ctypes.byref(st)),
                            "nxg_pagerank_adjoint", allow=(_lib.NXG_ENOTCONV,))
        out = st.as_dict()
        out["status"] = rc
        return lam, gw, gt, out


class WeightedPageRank(torch.autograd.Function):
    """x* = WeightedPageRank.apply(w, t, dsss, damping, tol, max_iters).

    Forward: stores w (input edge order) in the DSSS and iterates weighted
    PageRank in FP64 to ||x^{k+1} - x^k||_1 <= tol. Only x* is saved (with a
    reference to the input w, put back into the handle if another forward has
    stored other weights since). Backward:
    the hand-written adjoint over the transposed sub-shards returns dL/dw (the
    given weights, no renormalisation) and dL/dt. The DSSS must be built with
    weights, transpose=True, keep_perm=True.
    """

    @staticmethod
    def forward(ctx, w, t, dsss, damping=0.85, tol=1e-8, max_iters=100000):
        dsss.set_weights(w)
        x, st = dsss.pagerank(int(max_iters), damping=damping, dtype=torch.float64, tol=tol,
                              teleport=t, weighted=True)
        if st["status"] != _lib.NXG_OK:
            raise RuntimeError("weighted PageRank did not reach tol=%g in %d iterations"
                               % (tol, max_iters))
        # x* is the only computed state kept; w is the caller's own input, held
        # to restore the stored weights if the handle was given others since
        ctx.save_for_backward(x, w)
        ctx.dsss = dsss
        ctx.version = dsss.weights_version
        ctx.damping = damping
        ctx.adj_tol = min(tol, 1e-10)
        ctx.max_iters = max_iters
        ctx.w_dtype = w.dtype
        ctx.t_dtype = t.dtype if t is not None else None
        ctx.forward_stats = st
        return x

    @staticmethod
    def backward(ctx, gx):
        x, w = ctx.saved_tensors
        if ctx.dsss.weights_version != ctx.version:
            # another forward stored other weights in the handle: put these back
            ctx.dsss.set_weights(w)
            ctx.version = ctx.dsss.weights_version
        _, gw, gt, _ = ctx.dsss.pagerank_adjoint(x, gx, damping=ctx.damping, tol=ctx.adj_tol,
                                                 max_iters=ctx.max_iters)
        gt_out = gt.to(ctx.t_dtype) if ctx.t_dtype is not None else None
        return gw.to(ctx.w_dtype), gt_out, None, None, None, None


class MultiDSSS:
    """Many independent graphs iterated together: each iteration's edge work of all
    graphs is one launch."""

    def __init__(self, handle, device, sizes):
        self._h = handle
        self.device = device
        self.sizes = sizes  # vertex counts

    @classmethod
    def build(cls, graphs, interval=0, tile=0, chunk=0, order="dst", relabel=False, stream=None):
        """graphs: list of (src, dst, n) with int32 device tensors."""
        install_torch_allocator()
        keep = []
        descs = (_lib.BuildDesc * len(graphs))()
        for i, (src, dst, n) in enumerate(graphs):
            src = _dev_i32(src, "src")
            dst = _dev_i32(dst, "dst")
            keep += [src, dst]
            descs[i] = _lib.BuildDesc(n=int(n), m=src.numel(),
                                      d_src=src.data_ptr() if src.numel() else None,
                                      d_dst=dst.data_ptr() if dst.numel() else None,
                                      d_weight=None, interval=int(interval), tile=int(tile),
                                      chunk=int(chunk), value_bytes=0,
                                      flags=_lib.NXG_BUILD_RELABEL if relabel else 0,
                                      order={"dst": _lib.NXG_ORDER_DST, "src": _lib.NXG_ORDER_SRC}[order])
        h = ctypes.c_void_p()
        dev = graphs[0][0].device
        with torch.cuda.device(dev):
            _lib.check(_lib.lib().nxg_multi_build(len(graphs), descs, _stream_handle(stream),
                                                  ctypes.byref(h)), "nxg_multi_build")
        return cls(h, dev, [int(g[2]) for g in graphs])

    def close(self):
        if self._h:
            _lib.lib().nxg_multi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pagerank(self, iters, damping=0.85, persistent=False, out=None, capture=False):
        """x of every graph after iters iterations; out: optional list of FP32
        tensors [n_i] to write into (else views of one new buffer).
        capture=True records the run's launches into a hipGraph kept by the
        handle and replays it on later runs with the same iteration count and
        damping (the outputs may differ from run to run)."""
        if out is None:
            flat = torch.empty(sum(self.sizes), dtype=torch.float32, device=self.device)
            outs = list(flat.split(self.sizes))
        else:
            outs = list(out)
            if len(outs) != len(self.sizes) or any(
                    o.numel() != n or o.dtype != torch.float32 or not o.is_contiguous()
                    for o, n in zip(outs, self.sizes)):
                raise ValueError("out must hold one contiguous FP32 tensor [n_i] per graph")
        ptrs = (ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        d = _lib.RunDesc(program=_lib.NXG_PAGERANK, dtype=_lib.NXG_F32, batch=1,
                         damping=float(damping), max_iters=int(iters), tol=0.0, d_teleport=None,
                         roots=None, d_values=None,
                         flags=(_lib.NXG_RUN_PERSISTENT if persistent else 0) |
                         (_lib.NXG_RUN_CAPTURE if capture else 0), d_seeds=None)
        st = _lib.RunStats()
        with torch.cuda.device(self.device):
            _lib.check(_lib.lib().nxg_multi_run(self._h, ctypes.byref(d), ptrs, _stream_handle(),
                                                ctypes.byref(st)), "nxg_multi_run")
        return outs, st.as_dict()
