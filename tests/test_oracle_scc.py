"""Pins for the oracle's SCC (mutual reachability, label = smallest id of the
component): exhaustive brute force on every digraph with 4 vertices (self-loops
included) against a transitive closure, closed forms, and scipy's strong
components on R-MAT graphs."""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import oracle
import rmatgen

PAIRS = [(u, v) for u in range(4) for v in range(4)]


def _graph(mask):
    e = [PAIRS[b] for b in range(16) if mask >> b & 1]
    return (np.array([a for a, _ in e], np.int32), np.array([b for _, b in e], np.int32))


def _closure_labels(n, src, dst):
    # reach[i, j]: j is reachable from i (Warshall's closure; i reaches itself)
    reach = np.eye(n, dtype=bool)
    reach[src, dst] = True
    for k in range(n):
        reach |= reach[:, k:k + 1] & reach[k:k + 1, :]
    mutual = reach & reach.T
    return [int(np.flatnonzero(mutual[i])[0]) for i in range(n)]


def _canonical(labels):
    # any numbering of the components -> smallest member id
    lo = {}
    for v, c in enumerate(labels):
        lo[c] = min(lo.get(c, v), v)
    return np.array([lo[c] for c in labels], np.int32)


def _scipy_scc(n, src, dst):
    a = coo_matrix((np.ones(len(src)), (src, dst)), shape=(n, n)).tocsr()
    k, lab = connected_components(a, directed=True, connection="strong")
    return _canonical(lab.tolist()), k


def test_scc_every_4_vertex_digraph():
    for mask in range(1 << 16):
        src, dst = _graph(mask)
        lab, cnt = oracle.scc(4, src, dst)
        want = _closure_labels(4, src, dst)
        assert lab.tolist() == want, mask
        assert cnt == len(set(want))


def test_scc_random_small_graphs_against_closure():
    rng = np.random.default_rng(11)
    for trial in range(40):
        n = int(rng.integers(1, 60))
        m = int(rng.integers(0, 3 * n))
        src = rng.integers(0, n, m).astype(np.int32)
        dst = rng.integers(0, n, m).astype(np.int32)
        assert oracle.scc(n, src, dst)[0].tolist() == _closure_labels(n, src, dst)


def test_scc_closed_forms():
    n = 50
    v = np.arange(n, dtype=np.int32)
    # a directed cycle written from the top down: one component labelled 0
    lab, cnt = oracle.scc(n, (v + 1) % n, v)
    assert np.all(lab == 0) and cnt == 1
    # a DAG (every edge from a larger to a smaller id): all singletons
    a, b = np.triu_indices(n, 1)
    lab, cnt = oracle.scc(n, b.astype(np.int32), a.astype(np.int32))
    assert np.array_equal(lab, v) and cnt == n
    # two 3-cycles {7, 3, 9} and {1, 4, 2} joined by one edge 9 -> 1, in a
    # 12-vertex graph: the two cycles, everything else alone
    src = np.array([7, 3, 9, 1, 4, 2, 9], np.int32)
    dst = np.array([3, 9, 7, 4, 2, 1, 1], np.int32)
    lab, cnt = oracle.scc(12, src, dst)
    want = np.arange(12, dtype=np.int32)
    want[[3, 7, 9]] = 3
    want[[1, 2, 4]] = 1
    assert np.array_equal(lab, want) and cnt == 8
    # no edges at all
    lab, cnt = oracle.scc(5, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert np.array_equal(lab, np.arange(5)) and cnt == 5


def test_scc_of_symmetric_graph_is_wcc():
    src, dst = rmatgen.rmat_edges(10, 3, seed=9)
    s2 = np.concatenate([src, dst]).astype(np.int32)
    d2 = np.concatenate([dst, src]).astype(np.int32)
    assert np.array_equal(oracle.scc(1024, s2, d2)[0], oracle.wcc(1024, src, dst)[0])


@pytest.mark.parametrize("scale,ef,seed", [(10, 2, 3), (12, 4, 5), (14, 8, 6)])
def test_scc_rmat_against_scipy(scale, ef, seed):
    n = 1 << scale
    src, dst = rmatgen.rmat_edges(scale, ef, seed=seed)
    lab, cnt = oracle.scc(n, src, dst)
    want, k = _scipy_scc(n, src, dst)
    assert np.array_equal(lab, want) and cnt == k
