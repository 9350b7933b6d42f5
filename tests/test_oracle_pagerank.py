"""Pins for the oracle's PageRank: closed forms, invariants, and a dense-matrix
formulation solved with numpy (a different route to the same numbers)."""
import numpy as np
import pytest

import oracle
import rmatgen

D = 0.85


def _cycle(n):
    src = np.arange(n, dtype=np.int32)
    return src, (src + 1) % n


def _complete(n, loops):
    s, t = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = np.ones_like(s, dtype=bool) if loops else (s != t)
    return s[keep].astype(np.int32), t[keep].astype(np.int32)


def _dense_google(n, src, dst, w=None):
    """Column-stochastic iteration matrix G = d (M + (1/n) 1 1_D^T), M[v, u] = sum w_e."""
    deg = np.bincount(src, minlength=n)
    if w is None:
        w = 1.0 / deg[src]
    M = np.zeros((n, n))
    np.add.at(M, (dst, src), w)
    G = D * (M + np.outer(np.ones(n), (deg == 0).astype(float)) / n)
    return G


@pytest.mark.parametrize("name,edges", [
    ("cycle", _cycle(7)),
    ("complete", _complete(6, loops=False)),
    ("complete_loops", _complete(5, loops=True)),
    ("edgeless", (np.zeros(0, np.int32), np.zeros(0, np.int32))),
    ("regular3", (np.repeat(np.arange(9), 3).astype(np.int32),
                  ((np.repeat(np.arange(9), 3) + np.tile([1, 2, 4], 9)) % 9).astype(np.int32))),
])
def test_uniform_closed_forms(name, edges):
    n = int(max(edges[0].max(initial=-1), edges[1].max(initial=-1)) + 1) or 4
    for k in (1, 2, 5, 10):
        x, res = oracle.pagerank(n, *edges, iters=k)
        assert np.allclose(x, 1.0 / n, rtol=0, atol=1e-15), name
        assert np.all(res <= 1e-15)


def test_two_vertex_path_closed_form():
    src, dst = np.array([0], np.int32), np.array([1], np.int32)
    for k in range(0, 12):
        x, _ = oracle.pagerank(2, src, dst, iters=k)
        x0 = 1 / (2 + D) + (-D / 2) ** k * D / (2 * (2 + D))
        assert abs(x[0] - x0) < 1e-15 and abs(x[1] - (1 - x0)) < 1e-15


def test_in_star_fixed_point():
    n = 50
    src = np.arange(1, n, dtype=np.int32)
    dst = np.zeros(n - 1, dtype=np.int32)
    x, res = oracle.pagerank(n, src, dst, iters=500, tol=1e-16)
    hub = (1 + (n - 1) * D) / (n + (n - 1) * D)
    assert abs(x[0] - hub) < 1e-14
    assert np.allclose(x[1:], (D * hub + 1 - D) / n, atol=1e-15)


def test_mass_conserved_every_iteration():
    src, dst = rmatgen.rmat_edges(11, 8, seed=21)
    n = 2048
    deg = np.bincount(src, minlength=n)
    assert (deg == 0).any()          # the invariant must hold with dangling vertices
    for k in range(1, 8):
        x, _ = oracle.pagerank(n, src, dst, iters=k)
        assert abs(x.sum() - 1.0) < 1e-14


def test_dense_matrix_iteration_and_fixed_point():
    scale = 9
    n = 1 << scale
    src, dst = rmatgen.rmat_edges(scale, 6, seed=5)
    rng = np.random.default_rng(0)
    t = rng.random(n)
    t /= t.sum()
    G = _dense_google(n, src, dst)
    xk = t.copy()
    for k in range(1, 9):
        xk = G @ xk + (1 - D) * t
        x, res = oracle.pagerank(n, src, dst, iters=k, t=t)
        assert np.abs(x - xk).sum() < 1e-13
    xf = np.linalg.solve(np.eye(n) - G, (1 - D) * t)
    x, res = oracle.pagerank(n, src, dst, iters=1000, t=t, tol=1e-15)
    assert np.abs(x - xf).sum() < 1e-12
    assert len(res) < 1000 and res[-1] <= 1e-15


def test_weighted_dense_matrix():
    n = 300
    src, dst = rmatgen.rmat_edges(8, 8, seed=7)
    src = np.concatenate([src, np.array([299], np.int32)])
    dst = np.concatenate([dst, np.array([0], np.int32)])
    w = rmatgen.row_normalized_weights(src, n, seed=107).astype(np.float64)
    G = _dense_google(n, src, dst, w)
    t = np.full(n, 1.0 / n)
    xk = t.copy()
    for k in range(1, 6):
        xk = G @ xk + (1 - D) * t
    x, _ = oracle.pagerank(n, src, dst, iters=5, w=w)
    assert np.abs(x - xk).sum() < 1e-13


def test_personalized_superposition_and_warm_start():
    scale = 10
    n = 1 << scale
    src, dst = rmatgen.rmat_edges(scale, 8, seed=9)
    seeds = [3, 100, 517]
    alpha = np.array([0.5, 0.3, 0.2])
    cols = []
    for s in seeds:
        t = np.zeros(n)
        t[s] = 1.0
        x, _ = oracle.pagerank(n, src, dst, iters=12, t=t)
        assert abs(x.sum() - 1) < 1e-14
        cols.append(x)
    t = np.zeros(n)
    t[seeds] = alpha
    x, _ = oracle.pagerank(n, src, dst, iters=12, t=t)
    assert np.abs(x - np.stack(cols, 1) @ alpha).sum() < 1e-14
    # 12 iterations == 7 iterations, then 5 more started from that vector.
    x7, _ = oracle.pagerank(n, src, dst, iters=7, t=t)
    x12, _ = oracle.pagerank(n, src, dst, iters=5, t=t, x0=x7)
    assert np.array_equal(x12, x)


def test_duplicate_edges_and_self_loops_count_in_outdegree():
    # 0 -> 1 twice and 0 -> 0 once: vertex 0 sends 2/3 of its rank to 1, 1/3 to itself.
    src = np.array([0, 0, 0], np.int32)
    dst = np.array([1, 1, 0], np.int32)
    x, _ = oracle.pagerank(2, src, dst, iters=1)
    # delta = x_1 = 1/2 (vertex 1 dangling)
    assert abs(x[0] - (D * (0.5 / 3 + 0.25) + (1 - D) / 2)) < 1e-15
    assert abs(x[1] - (D * (0.5 * 2 / 3 + 0.25) + (1 - D) / 2)) < 1e-15


def test_invalid_input_rejected():
    with pytest.raises(ValueError):
        oracle.pagerank(4, np.array([0], np.int32), np.array([4], np.int32), iters=1)
