"""Weighted-PageRank adjoint on the GPU against the FP64 oracle gradient, the
Euler identity and central finite differences; the autograd Function."""
import numpy as np
import pytest
import torch

import oracle
import rmatgen
from paper_1510_06916_amd import DSSS, WeightedPageRank
from gpu_util import rel_l1, say, to_dev

pytestmark = pytest.mark.gpu
D = 0.85


def _problem(scale, ef, seed, device, interval=None, order="dst"):
    n = 1 << scale
    src, dst = rmatgen.rmat_edges(scale, ef, seed)
    w = rmatgen.row_normalized_weights(src, n, seed=seed + 100)
    g = rmatgen.normal_f32(seed + 200, n).astype(np.float64)
    dsss = DSSS.build(to_dev(src, device), to_dev(dst, device), n, interval=interval,
                      weights=torch.from_numpy(w), transpose=True, keep_perm=True, order=order)
    return n, src, dst, w, g, dsss


@pytest.mark.parametrize("scale,interval,order", [(10, 256, "dst"), (12, None, "dst"),
                                                  (12, 512, "src")])
def test_adjoint_matches_oracle(gpu_device, scale, interval, order):
    n, src, dst, w, g, dsss = _problem(scale, 8, 30 + scale, gpu_device, interval, order)
    w64 = w.astype(np.float64)
    xs, _ = oracle.pagerank(n, src, dst, iters=5000, w=w64, tol=1e-15)
    lam_o, gw_o, gt_o, it_o = oracle.pagerank_adjoint(n, src, dst, w64, xs, g, tol=1e-14)
    lam, gw, gt, st = dsss.pagerank_adjoint(torch.from_numpy(xs), torch.from_numpy(g), tol=1e-14)
    say("adjoint scale=%d: oracle %d its, gpu %d its" % (scale, it_o, st["iterations"]))
    assert st["converged"] == 1
    assert rel_l1(lam.cpu().numpy(), lam_o) <= 1e-11
    assert rel_l1(gt.cpu().numpy(), gt_o) <= 1e-11
    assert rel_l1(gw.cpu().numpy(), gw_o) <= 1e-6   # FP32 output


def test_function_forward_backward_and_euler(gpu_device):
    n, src, dst, w, g, dsss = _problem(11, 8, 61, gpu_device)
    rng = np.random.default_rng(0)
    t = rng.random(n)
    t /= t.sum()
    wt = torch.from_numpy(w).to(gpu_device).requires_grad_(True)
    tt = torch.from_numpy(t).to(gpu_device).requires_grad_(True)
    x = WeightedPageRank.apply(wt, tt, dsss, D, 1e-13)
    ref, _ = oracle.pagerank(n, src, dst, iters=5000, w=w.astype(np.float64), t=t, tol=1e-15)
    assert rel_l1(x.detach().cpu().numpy(), ref) <= 1e-11
    L = (x * torch.from_numpy(g).to(gpu_device)).sum()
    L.backward()
    _, gw_o, gt_o, _ = oracle.pagerank_adjoint(n, src, dst, w.astype(np.float64), ref, g, tol=1e-14)
    assert rel_l1(wt.grad.cpu().numpy(), gw_o) <= 1e-6
    assert rel_l1(tt.grad.cpu().numpy(), gt_o) <= 1e-10
    # x* is linear in t: L = sum_v t_v dL/dt_v
    Lv = float(L.detach())
    assert abs(Lv - float((tt.detach() * tt.grad).sum())) <= 1e-12 * max(1.0, abs(Lv))


def test_finite_differences_small(gpu_device):
    n, src, dst, w, g, dsss = _problem(9, 8, 71, gpu_device)
    gd = torch.from_numpy(g).to(gpu_device)
    wt = torch.from_numpy(w).to(gpu_device)
    x = WeightedPageRank.apply(wt, None, dsss, D, 1e-14)
    _, gw, _, _ = dsss.pagerank_adjoint(x, gd, tol=1e-14)
    gw = gw.cpu().numpy().astype(np.float64)
    h = 1e-3
    picks = np.random.default_rng(3).choice(len(src), 20, replace=False)
    fd = []
    for e in picks:
        wp, wm = wt.clone(), wt.clone()
        wp[e] += h
        wm[e] -= h
        lp = float((WeightedPageRank.apply(wp, None, dsss, D, 1e-14) * gd).sum())
        lm = float((WeightedPageRank.apply(wm, None, dsss, D, 1e-14) * gd).sum())
        # the FP32 weights make the perturbation h_eff = fl(w+h) - fl(w-h)
        he = float(np.float32(w[e] + h)) - float(np.float32(w[e] - h))
        fd.append((lp - lm) / he)
    fd = np.array(fd)
    assert np.linalg.norm(fd - gw[picks]) <= 1e-4 * np.linalg.norm(fd)


def test_adjoint_requires_transpose(gpu_device):
    src, dst = rmatgen.rmat_edges(8, 4, seed=1)
    w = rmatgen.row_normalized_weights(src, 256, seed=2)
    dsss = DSSS.build(to_dev(src, gpu_device), to_dev(dst, gpu_device), 256,
                      weights=torch.from_numpy(w))
    with pytest.raises(Exception, match="EINVAL"):
        dsss.pagerank_adjoint(torch.zeros(256, dtype=torch.float64), torch.ones(256, dtype=torch.float64))
