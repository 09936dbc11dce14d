"""rbf_matvec_device_noalloc, the allocation-free form of rbf_matvec_device
(original order), through the C ABI (-m gpu).

Its product must equal rbf_matvec_device's bit for bit (the same kernels; only
the staging of the sorted-order vectors moves to the library's fixed device
array), on two calls in a row, the second with fewer points than the first,
in both precisions, and the FP64 product must meet the oracle's bar.  The call
takes nothing from the library's block cache, and a problem above the fixed
array's size is refused with RBF_ELIMIT.
"""
import sys

import numpy as np
import pytest

import paper_0909_5413_amd as R
from paper_0909_5413_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    R.lib()
    return torch


def test_noalloc_matvec_equals_allocating_form(torch_dev, oracle_mod):
    torch = torch_dev
    st = torch.cuda.current_stream()
    big = W.Workload("noalloc_big", 230, 0.8, seed=611)       # 52,900 points
    small = W.Workload("noalloc_small", 37, 0.9, seed=612)    # 1,369 points
    for w in (big, small):            # two calls in a row, the second smaller
        pts = w.points()
        say("noalloc", w.name, w.n)
        h = R.rbf_setup(pts, w.values(pts), w.sigma, w.cutoff, w.overlap)
        try:
            wv = W.random_weights(w.n, 613)
            dw = torch.tensor(wv, device="cuda", dtype=torch.float64)
            for prec in (R.RBF_FP64, R.RBF_MIXED):
                ref = torch.empty_like(dw)
                R.rbf_matvec_device(h, dw, ref, prec, R.RBF_ORDER_ORIGINAL, st)
                torch.cuda.synchronize()
                idle = R.rbf_block_cache(-1)
                got = torch.full_like(dw, float("nan"))
                R.rbf_matvec_device_noalloc(h, dw, got, prec, st)
                torch.cuda.synchronize()
                assert R.rbf_block_cache(-1) == idle
                assert torch.equal(got, ref), (w.name, prec)
                if prec == R.RBF_FP64:
                    P = oracle_mod.Problem(pts, w.sigma, w.cutoff, w.overlap)
                    yo = P.matvec(wv)
                    scale = P.matvec(np.abs(wv))
                    P.close()
                    err = np.abs(got.cpu().numpy() - yo) / scale
                    assert err.max() <= 1e-13, err.max()
        finally:
            R.rbf_destroy(h)


def test_noalloc_matvec_size_limit(torch_dev):
    torch = torch_dev
    side = 2049                      # 4,198,401 points > RBF_NOALLOC_MAX_POINTS
    assert side * side > R.RBF_NOALLOC_MAX_POINTS
    w = W.Workload("noalloc_limit", side, 1.0, seed=614)
    pts = w.points()
    say("noalloc limit", w.n)
    d_pts = torch.tensor(pts, device="cuda")
    h = R.rbf_setup_device(d_pts, None, w.n, w.sigma, w.cutoff, w.overlap,
                           torch.cuda.current_stream())
    try:
        dw = torch.zeros(w.n, device="cuda", dtype=torch.float64)
        dy = torch.empty_like(dw)
        with pytest.raises(R.RbfError) as e:
            R.rbf_matvec_device_noalloc(h, dw, dy, R.RBF_FP64, torch.cuda.current_stream())
        assert e.value.status == R.RBF_ELIMIT
    finally:
        torch.cuda.synchronize()
        R.rbf_destroy(h)
