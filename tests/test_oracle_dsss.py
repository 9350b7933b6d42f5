"""Pins for the oracle's DSSS edge order: the paper's worked example and the
layout invariants of Sec. II-A / Sec. III-A on random graphs."""
import os

import numpy as np

import oracle
import rmatgen

HERE = os.path.dirname(os.path.abspath(__file__))


def load_fig1():
    meta, edges = {}, []
    with open(os.path.join(HERE, "golden", "fig1_subshard_3_2.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            a, b = line.split()
            if a.isdigit():
                edges.append((int(a), int(b)))
            else:
                meta[a] = int(b)
    return meta, edges


def test_paper_example_subshard_order():
    meta, want = load_fig1()
    I = meta["interval_size"]
    # the three edges of the example plus edges in other sub-shards, shuffled
    edges = want + [(0, 1), (1, 0), (2, 5), (3, 5), (6, 7), (7, 2), (4, 4), (5, 0), (0, 3)]
    rng = np.random.default_rng(0)
    order = rng.permutation(len(edges))
    src = np.array([edges[k][0] for k in order], np.int32)
    dst = np.array([edges[k][1] for k in order], np.int32)
    n = 8
    perm, off = oracle.dsss_order(n, src, dst, I)
    P = n // I
    s = meta["destination_interval"] * P + meta["source_interval"]
    got = [(int(src[perm[k]]), int(dst[perm[k]])) for k in range(off[s], off[s + 1])]
    assert got == want


def test_dsss_invariants_random():
    n = 1000
    src, dst = rmatgen.rmat_edges(10, 8, seed=12)
    keep = (src < n) & (dst < n)
    src, dst = src[keep], dst[keep]
    rng = np.random.default_rng(4)
    # shuffled input with a few duplicated edges to exercise the stable tie rule
    dup = rng.choice(len(src), 50, replace=False)
    src = np.concatenate([src, src[dup]])
    dst = np.concatenate([dst, dst[dup]])
    p = rng.permutation(len(src))
    src, dst = src[p], dst[p]
    for I in (1, 7, 64, 250, 1000, 4096):
        P = -(-n // I)
        perm, off = oracle.dsss_order(n, src, dst, I)
        assert sorted(perm.tolist()) == list(range(len(src)))
        assert off[0] == 0 and off[-1] == len(src) and np.all(np.diff(off) >= 0)
        s_, d_ = src[perm], dst[perm]
        for j in range(P):
            for i in range(P):
                a, b = off[j * P + i], off[j * P + i + 1]
                if a == b:
                    continue
                assert np.all(s_[a:b] // I == i) and np.all(d_[a:b] // I == j)
                key = d_[a:b].astype(np.int64) * n + s_[a:b]
                assert np.all(np.diff(key) >= 0)
                ties = np.diff(key) == 0
                assert np.all(np.diff(perm[a:b])[ties] > 0)
