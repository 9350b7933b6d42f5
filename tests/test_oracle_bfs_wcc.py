"""Pins for the oracle's BFS and WCC: exhaustive brute force on every digraph with
4 vertices (self-loops included) against textbook algorithms, plus closed forms."""
from collections import deque

import numpy as np
import pytest

import oracle
import rmatgen

INF = oracle.INF
PAIRS = [(u, v) for u in range(4) for v in range(4)]


def _graph(mask):
    e = [PAIRS[b] for b in range(16) if mask >> b & 1]
    return (np.array([a for a, _ in e], np.int32), np.array([b for _, b in e], np.int32))


def _queue_bfs(n, src, dst, root):
    adj = [[] for _ in range(n)]
    for a, b in zip(src, dst):
        adj[a].append(b)
    lev = [INF] * n
    lev[root] = 0
    q = deque([root])
    while q:
        u = q.popleft()
        for v in adj[u]:
            if lev[v] == INF:
                lev[v] = lev[u] + 1
                q.append(v)
    return lev


def _union_find(n, src, dst):
    p = list(range(n))

    def find(a):
        while p[a] != a:
            p[a] = p[p[a]]
            a = p[a]
        return a
    for a, b in zip(src, dst):
        ra, rb = find(a), find(b)
        if ra != rb:
            p[max(ra, rb)] = min(ra, rb)
    return [min(v for v in range(n) if find(v) == find(u)) for u in range(n)]


def test_bfs_every_4_vertex_digraph():
    for mask in range(1 << 16):
        src, dst = _graph(mask)
        for root in range(4):
            lev, rounds, mx = oracle.bfs(4, src, dst, root)
            want = _queue_bfs(4, src, dst, root)
            assert lev.tolist() == want, (mask, root)
            finite = [x for x in want if x != INF]
            assert mx == max(finite)
            # one synchronous round reaches exactly one more level
            assert rounds == mx


def test_wcc_every_4_vertex_digraph():
    for mask in range(1 << 16):
        src, dst = _graph(mask)
        lab, rounds = oracle.wcc(4, src, dst)
        assert lab.tolist() == _union_find(4, src, dst), mask


def test_bfs_path_and_unreachable():
    n = 40
    src = np.arange(n - 2, dtype=np.int32)     # path 0 -> 1 -> ... -> n-2 ; n-1 isolated
    lev, rounds, mx = oracle.bfs(n, src, src + 1, 0)
    assert lev[:n - 1].tolist() == list(range(n - 1)) and lev[n - 1] == INF
    assert rounds == n - 2 and mx == n - 2
    lev, rounds, _ = oracle.bfs(n, src, src + 1, n - 1)
    assert lev[n - 1] == 0 and np.all(lev[:n - 1] == INF) and rounds == 0


def test_bfs_wcc_random_graphs_against_textbook():
    rng = np.random.default_rng(3)
    for trial in range(30):
        n = int(rng.integers(2, 64))
        m = int(rng.integers(0, 3 * n))
        src = rng.integers(0, n, m).astype(np.int32)
        dst = rng.integers(0, n, m).astype(np.int32)
        root = int(rng.integers(0, n))
        assert oracle.bfs(n, src, dst, root)[0].tolist() == _queue_bfs(n, src, dst, root)
        assert oracle.wcc(n, src, dst)[0].tolist() == _union_find(n, src, dst)


def test_wcc_known_components():
    # two cliques {0..4} and {5..9} written with edges pointing "down" only, a path
    # 10-11-...-19 written backwards, and an isolated vertex 20.
    src, dst = [], []
    for base in (0, 5):
        for a in range(5):
            for b in range(a):
                src.append(base + a)
                dst.append(base + b)
    for v in range(11, 20):
        src.append(v)
        dst.append(v - 1)
    lab, rounds = oracle.wcc(21, np.array(src, np.int32), np.array(dst, np.int32))
    assert lab.tolist() == [0] * 5 + [5] * 5 + [10] * 10 + [20]
    assert rounds == 9          # label 10 walks one hop per round down the path


def test_rmat_wcc_is_a_partition_fixed_point():
    src, dst = rmatgen.rmat_edges(10, 4, seed=2)
    lab, _ = oracle.wcc(1024, src, dst)
    assert np.all(lab[src] == lab[dst])
    assert np.all(lab <= np.arange(1024)) and np.all(lab[lab] == lab)
