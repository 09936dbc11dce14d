"""Graph launches of the Arnoldi step against single launches (-m gpu).

The Gram-Schmidt work of each Arnoldi step (Section 2.2's GMRES iteration) is
captured once per step index as a HIP graph and replayed.  A captured graph is
replayed many times per solve and across solves; these tests replay it with
the program's own eager work and synchronisations in between, on the default
stream and on a side stream, and check every solve bit for bit against the
same solve with the kernels launched one by one, and against the oracle's
residual.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_0909_5413_amd as R
from paper_0909_5413_amd import workloads as W
from tests.gates import residual_gate

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


def solve(torch, h, n, prec, rtol, stream):
    lam = torch.empty(n, device="cuda", dtype=torch.float64)
    opts = R.default_opts(rtol=rtol, precision=prec, stream=stream)
    info, _ = R.rbf_solve_device(h, lam, opts)
    torch.cuda.synchronize()
    return lam.cpu().numpy(), info.iterations


@pytest.mark.parametrize("prec", [R.RBF_FP64, R.RBF_MIXED])
def test_graph_replays_match_single_launches(torch_dev, prec):
    torch = torch_dev
    w = W.MINI
    pts = w.points()
    f = w.values(pts)
    say("graph replays", w.name, "precision", prec)
    d_pts = torch.tensor(pts, device="cuda")
    d_f = torch.tensor(f, device="cuda")
    side = torch.cuda.Stream()
    h = R.rbf_setup_device(d_pts, d_f, w.n, w.sigma, w.cutoff, w.overlap,
                           torch.cuda.current_stream())
    try:
        R.rbf_set_graphs(h, False)
        ref, it_ref = solve(torch, h, w.n, prec, 1e-12, torch.cuda.current_stream())
        R.rbf_set_graphs(h, True)
        rng = np.random.default_rng(7)
        for rep in range(4):
            # eager work of the program between replays
            v = torch.tensor(rng.uniform(-1, 1, w.n), device="cuda")
            y = torch.empty_like(v)
            R.rbf_matvec_device(h, v, y, R.RBF_FP64, R.RBF_ORDER_SORTED,
                                torch.cuda.current_stream())
            z = (y * 2.0).sum().item()
            assert np.isfinite(z)
            st = torch.cuda.current_stream() if rep % 2 == 0 else side
            with torch.cuda.stream(st):
                got, it = solve(torch, h, w.n, prec, 1e-12, st)
            say("replay", rep, "iterations", it)
            assert it == it_ref
            assert np.array_equal(got, ref), np.max(np.abs(got - ref))
        P = oracle.Problem(pts, w.sigma, w.cutoff, w.overlap)
        assert P.rel_residual(f, ref) <= residual_gate(P, f, ref, 1e-12)
        # and single launches again after the graphs ran
        R.rbf_set_graphs(h, False)
        again, _ = solve(torch, h, w.n, prec, 1e-12, torch.cuda.current_stream())
        assert np.array_equal(again, ref)
    finally:
        R.rbf_destroy(h)


def test_graphs_rebuilt_for_larger_restart(torch_dev):
    """A larger restart length reallocates the Krylov basis; the captured
    steps refer to the old one and must be rebuilt, not replayed."""
    torch = torch_dev
    w = W.MINI
    pts = w.points()
    f = w.values(pts)
    say("restart change", w.name)
    h = R.rbf_setup(pts, f, w.sigma, w.cutoff, w.overlap)
    try:
        out = {}
        for use in (False, True):
            R.rbf_set_graphs(h, use)
            for m in (10, 30, 20):
                lam, info, _ = R.rbf_solve(h, w.n, R.default_opts(rtol=1e-12, restart=m))
                out[(use, m)] = (lam, info.iterations)
        for m in (10, 30, 20):
            assert out[(True, m)][1] == out[(False, m)][1]
            assert np.array_equal(out[(True, m)][0], out[(False, m)][0])
    finally:
        R.rbf_destroy(h)
