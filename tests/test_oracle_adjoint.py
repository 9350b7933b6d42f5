"""Pins for the oracle's weighted-PageRank adjoint: a dense torch formulation
differentiated by autograd, the Euler identity, and central finite differences."""
import numpy as np
import torch

import oracle
import rmatgen

D = 0.85


def _graph(scale, ef, seed, n):
    src, dst = rmatgen.rmat_edges(scale, ef, seed)
    w = rmatgen.row_normalized_weights(src, n, seed=seed + 100).astype(np.float64)
    return src, dst, w


def _dense_loss(n, src, dst, w_t, t_t, g_t):
    deg = np.bincount(src, minlength=n)
    M = torch.zeros((n, n), dtype=torch.float64)
    M = M.index_put((torch.from_numpy(dst).long(), torch.from_numpy(src).long()), w_t,
                    accumulate=True)
    dang = torch.from_numpy((deg == 0).astype(np.float64))
    G = D * (M + torch.outer(torch.ones(n, dtype=torch.float64), dang) / n)
    x = torch.linalg.solve(torch.eye(n, dtype=torch.float64) - G, (1 - D) * t_t)
    return (g_t * x).sum(), x


def test_adjoint_matches_dense_autograd():
    n = 256
    src, dst, w = _graph(8, 6, 31, n)
    g = rmatgen.normal_f32(231, n).astype(np.float64)
    t = np.full(n, 1.0 / n)
    w_t = torch.tensor(w, requires_grad=True)
    t_t = torch.tensor(t, requires_grad=True)
    L, x = _dense_loss(n, src, dst, w_t, t_t, torch.from_numpy(g))
    L.backward()
    lam, gw, gt, it = oracle.pagerank_adjoint(n, src, dst, w, x.detach().numpy(), g, tol=1e-14)
    assert it > 10
    ref_w = w_t.grad.numpy()
    ref_t = t_t.grad.numpy()
    assert np.abs(gw - ref_w).max() <= 1e-12 * np.abs(ref_w).max()
    assert np.abs(gt - ref_t).max() <= 1e-12 * np.abs(ref_t).max()


def test_euler_identity_and_ppr_symmetry():
    # x* is linear in t, so L = g.x* = sum_v t_v dL/dt_v; with g = e_j,
    # dL/dt_v = x*(e_v)_j (the j-th entry of the PageRank seeded at v).
    n = 512
    src, dst, w = _graph(9, 8, 41, n)
    rng = np.random.default_rng(1)
    t = rng.random(n)
    t /= t.sum()
    g = rmatgen.normal_f32(241, n).astype(np.float64)
    x, _ = oracle.pagerank(n, src, dst, iters=2000, w=w, t=t, tol=1e-16)
    _, _, gt, _ = oracle.pagerank_adjoint(n, src, dst, w, x, g, tol=1e-15)
    L = float(g @ x)
    assert abs(L - float(t @ gt)) < 1e-13 * max(1.0, abs(L))
    j = 17
    e_j = np.zeros(n)
    e_j[j] = 1.0
    _, _, gt_j, _ = oracle.pagerank_adjoint(n, src, dst, w, x, e_j, tol=1e-15)
    for v in (0, 5, 300):
        tv = np.zeros(n)
        tv[v] = 1.0
        xv, _ = oracle.pagerank(n, src, dst, iters=2000, w=w, t=tv, tol=1e-17)
        assert abs(gt_j[v] - xv[j]) < 1e-13


def test_central_finite_differences():
    n = 128
    src, dst, w = _graph(7, 8, 51, n)
    g = rmatgen.normal_f32(251, n).astype(np.float64)

    def loss(wv):
        x, _ = oracle.pagerank(n, src, dst, iters=400, w=wv, tol=0.0)
        return float(g @ x)

    x, _ = oracle.pagerank(n, src, dst, iters=400, w=w, tol=0.0)
    _, gw, _, _ = oracle.pagerank_adjoint(n, src, dst, w, x, g, tol=1e-15)
    h = 1e-4
    picks = np.random.default_rng(2).choice(len(src), 25, replace=False)
    fd = []
    for e in picks:
        wp, wm = w.copy(), w.copy()
        wp[e] += h
        wm[e] -= h
        fd.append((loss(wp) - loss(wm)) / (2 * h))
    fd = np.array(fd)
    # the central-difference error is O(h^2) times the third derivative of L in
    # one weight, far below the 1e-6 relative bound at h = 1e-4.
    assert np.linalg.norm(fd - gw[picks]) <= 1e-6 * np.linalg.norm(fd)
