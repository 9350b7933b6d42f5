"""CPU ORACLE -- test infrastructure only.

A plain single-threaded FP64 C implementation (oracle.c) of what the GPU path
computes, reached through ctypes. Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package. It shares no code with
the GPU library and never imports it.

Functions follow the paper (Chi et al., "NXgraph", 2015): PageRank by
synchronous iteration (Alg. 1, Sec. II-B, Sec. III-B1), BFS (Algs. 2-4), WCC
by minimum-label propagation on the symmetrised graph (Sec. II-A, Sec. IV-D),
SCC by its definition (mutual reachability; named in Sec. IV-D), the DSSS edge order (Sec. II-A, Sec. III-A), plus the adjoint of weighted
PageRank (not in the paper: the gradient of g^T x* at the fixed point).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
INF = np.iinfo(np.int32).max

_lib = None


def build():
    """Compile oracle.c with gcc (plain -O2, no vectorisation flags, no threads)."""
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", _SO,
                           os.path.join(_HERE, "oracle.c"), "-lm"])


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        i64, p, dbl = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double
        lib.orc_outdeg.argtypes = [i64, i64, p, p]
        lib.orc_pagerank.argtypes = [i64, i64, p, p, p, p, p, dbl, i64, dbl, p, p, p]
        lib.orc_bfs.argtypes = [i64, i64, p, p, ctypes.c_int32, p, p, p]
        lib.orc_wcc.argtypes = [i64, i64, p, p, p, p]
        lib.orc_pagerank_adjoint.argtypes = [i64, i64, p, p, p, p, p, dbl, dbl, i64, p, p, p, p]
        lib.orc_dsss_order.argtypes = [i64, i64, p, p, i64, p, p]
        lib.orc_scc.argtypes = [i64, i64, p, p, p, p]
        for f in (lib.orc_outdeg, lib.orc_pagerank, lib.orc_bfs, lib.orc_wcc,
                  lib.orc_pagerank_adjoint, lib.orc_dsss_order, lib.orc_scc):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _edges(src, dst):
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if src.shape != dst.shape or src.ndim != 1:
        raise ValueError("src and dst must be 1-D arrays of equal length")
    return src, dst


def _ptr(a):
    return None if a is None else a.ctypes.data


def _check(rc, what):
    if rc != 0:
        raise ValueError("%s: invalid input (code %d)" % (what, rc))


def outdeg(n, src):
    src = np.ascontiguousarray(src, dtype=np.int32)
    deg = np.empty(int(n), dtype=np.int64)
    _check(_L().orc_outdeg(int(n), len(src), _ptr(src), _ptr(deg)), "outdeg")
    return deg


def pagerank(n, src, dst, iters, d=0.85, w=None, t=None, tol=0.0, x0=None):
    """Returns (x, residuals) with x the FP64 vector after the iterations run."""
    src, dst = _edges(src, dst)
    n = int(n)
    wd = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    td = None if t is None else np.ascontiguousarray(t, dtype=np.float64)
    xd = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    x = np.empty(n, dtype=np.float64)
    res = np.empty(max(int(iters), 1), dtype=np.float64)
    done = ctypes.c_int64(0)
    rc = _L().orc_pagerank(n, len(src), _ptr(src), _ptr(dst), _ptr(wd), _ptr(td), _ptr(xd),
                           float(d), int(iters), float(tol), _ptr(x), _ptr(res),
                           ctypes.byref(done))
    _check(rc, "pagerank")
    return x, res[:done.value].copy()


def bfs(n, src, dst, root):
    """Returns (levels int32 with INF = unreachable, rounds, max finite level)."""
    src, dst = _edges(src, dst)
    lev = np.empty(int(n), dtype=np.int32)
    rounds = ctypes.c_int64(0)
    mx = ctypes.c_int32(0)
    rc = _L().orc_bfs(int(n), len(src), _ptr(src), _ptr(dst), int(root), _ptr(lev),
                      ctypes.byref(rounds), ctypes.byref(mx))
    _check(rc, "bfs")
    return lev, int(rounds.value), int(mx.value)


def wcc(n, src, dst):
    """Returns (labels int32 = smallest vertex id of the component, rounds)."""
    src, dst = _edges(src, dst)
    lab = np.empty(int(n), dtype=np.int32)
    rounds = ctypes.c_int64(0)
    rc = _L().orc_wcc(int(n), len(src), _ptr(src), _ptr(dst), _ptr(lab), ctypes.byref(rounds))
    _check(rc, "wcc")
    return lab, int(rounds.value)


def scc(n, src, dst):
    """Returns (labels int32 = smallest vertex id of the strongly connected
    component, number of components)."""
    src, dst = _edges(src, dst)
    lab = np.empty(int(n), dtype=np.int32)
    cnt = ctypes.c_int64(0)
    rc = _L().orc_scc(int(n), len(src), _ptr(src), _ptr(dst), _ptr(lab), ctypes.byref(cnt))
    _check(rc, "scc")
    return lab, int(cnt.value)


def pagerank_adjoint(n, src, dst, w, xstar, g, d=0.85, tol=1e-10, max_iters=100000):
    """Returns (lambda, dL/dw in input edge order, dL/dt, iterations)."""
    src, dst = _edges(src, dst)
    n = int(n)
    wd = np.ascontiguousarray(w, dtype=np.float64)
    xs = np.ascontiguousarray(xstar, dtype=np.float64)
    gd = np.ascontiguousarray(g, dtype=np.float64)
    lam = np.empty(n, dtype=np.float64)
    gw = np.empty(len(src), dtype=np.float64)
    gt = np.empty(n, dtype=np.float64)
    it = ctypes.c_int64(0)
    rc = _L().orc_pagerank_adjoint(n, len(src), _ptr(src), _ptr(dst), _ptr(wd), _ptr(xs),
                                   _ptr(gd), float(d), float(tol), int(max_iters), _ptr(lam),
                                   _ptr(gw), _ptr(gt), ctypes.byref(it))
    _check(rc, "pagerank_adjoint")
    return lam, gw, gt, int(it.value)


def dsss_order(n, src, dst, interval):
    """Returns (perm, offsets): perm[k] = input index of the k-th edge in DSSS order,
    offsets[j * P + i] = first position of sub-shard SS_{i.j} (P*P + 1 entries)."""
    src, dst = _edges(src, dst)
    n, interval = int(n), int(interval)
    P = (n + interval - 1) // interval
    perm = np.empty(len(src), dtype=np.int64)
    off = np.empty(P * P + 1, dtype=np.int64)
    rc = _L().orc_dsss_order(n, len(src), _ptr(src), _ptr(dst), interval, _ptr(perm), _ptr(off))
    _check(rc, "dsss_order")
    return perm, off
