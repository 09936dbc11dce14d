"""The interpolant on a regular lattice of targets (remeshing onto a lattice,
Sections 1 and 5; eq. rbf1 without the polynomial part) through the C ABI
(-m gpu), against the oracle's evaluation at the same coordinates (each
x0 + a * hx, one rounding per operation, as the library forms them).

Bar per target, 2 (k + 40) u (|A| |lambda|)_i with k its in-cutoff count:
both sides add at most k terms; a GPU term is w exp(-dx^2/2s^2) exp(-dy^2/2s^2)
(two table exponentials within 4.7 u each, the rounding of dx^2 and of dy^2
moving their arguments by at most x u with x = d2/(2 sigma^2) <= 18 inside the
cutoff, the weight product and the fused update), at most (11.4 + 18) u
relative; an oracle term exp(-d2/2s^2) with d2, its scaling, libm's exp, the
normalisation and the weight, at most (4 + 2 * 18) u.  Targets with no source
in the cutoff must give exactly 0.  The lattice path also agrees with
rbf_evaluate at the same points to the same bar, the host and device forms
agree bit for bit, and a box-truncated handle's lattice evaluation is the box
evaluation at those points, bit for bit.
"""
import sys

import numpy as np
import pytest

import paper_0909_5413_amd as R
from paper_0909_5413_amd import workloads as W
from tests.gates import U64

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


@pytest.fixture(scope="module")
def solved(torch_dev, oracle_mod):
    w = W.C0
    pts = w.points()
    f = w.values(pts)
    h = R.rbf_setup(pts, f, w.sigma, w.cutoff, 1)
    lam, info, st = R.rbf_solve(h, pts.shape[0], R.default_opts(rtol=1e-10))
    assert st == R.RBF_OK
    P = oracle_mod.Problem(pts, w.sigma, w.cutoff, 1)
    yield h, P, pts, lam, w
    R.rbf_destroy(h)


def lattice(x0, y0, hx, hy, nx, ny):
    ax = x0 + np.arange(nx, dtype=np.float64) * hx
    ay = y0 + np.arange(ny, dtype=np.float64) * hy
    gx, gy = np.meshgrid(ax, ay, indexing="xy")
    return np.ascontiguousarray(np.stack([gx.ravel(), gy.ravel()], axis=1))


def lattices(w):
    h = w.h
    return {
        # midway between the nodes (the remeshing lattice of the benchmark)
        "staggered": (-1.0 + h, -1.0 + h, h, h, w.n_side - 1, w.n_side - 1),
        # finer than the cells (several chunks per cell), reaching past the
        # nodes on every side (clamped cells, far targets with no source)
        "fine_wide": (-1.3, -1.1 - 0.37 * h, 0.31 * h, 0.53 * h, 260, 170),
        # coarser than the cells (cells without a column), uneven spacings
        "coarse": (-0.97, -1.02, 7.3 * w.sigma, 11.1 * w.sigma, 29, 19),
        "one_point": (0.1234, -0.4321, 1.0, 1.0, 1, 1),
        # a single row and a single column crossing the grid and its border
        "one_row": (-1.2, 0.0137, 0.6 * h, 1.0, 137, 1),
        "one_col": (0.271, -1.15, 1.0, 0.8 * h, 1, 93),
    }


@pytest.mark.parametrize("name", ["staggered", "fine_wide", "coarse", "one_point", "one_row",
                                  "one_col"])
def test_lattice_matches_oracle(torch_dev, solved, name):
    h, P, pts, lam, w = solved
    x0, y0, hx, hy, nx, ny = lattices(w)[name]
    tg = lattice(x0, y0, hx, hy, nx, ny)
    s = R.rbf_evaluate_lattice(h, x0, y0, hx, hy, nx, ny).ravel()
    so, cnt = P.evaluate(lam, tg, with_counts=True)
    scale = P.evaluate(np.abs(lam), tg)
    bar = 2 * (cnt + 40) * U64 * scale
    err = np.abs(s - so)
    worst = float((err[scale > 0] / bar[scale > 0]).max()) if np.any(scale > 0) else 0.0
    say("lattice", name, nx, "x", ny, "worst error / bar", worst, "empty targets",
        int((cnt == 0).sum()))
    assert np.all(err <= bar)
    assert np.all(s[cnt == 0] == 0.0)
    # the arbitrary-target path at the same coordinates
    st = R.rbf_evaluate(h, tg)
    assert np.all(np.abs(st - s) <= bar)
    # the device form, bit for bit
    d = torch_dev.empty(nx * ny, device="cuda", dtype=torch_dev.float64)
    R.rbf_evaluate_lattice_device(h, x0, y0, hx, hy, nx, ny, d, torch_dev.cuda.current_stream())
    torch_dev.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy(), s)


def test_lattice_errors(torch_dev, solved, oracle_mod):
    h, P, pts, lam, w = solved
    for bad in ((0.0, 0.0, 0.0, 0.1, 4, 4), (0.0, 0.0, 0.1, -0.1, 4, 4),
                (float("nan"), 0.0, 0.1, 0.1, 4, 4), (0.0, float("inf"), 0.1, 0.1, 4, 4),
                (0.0, 0.0, 1e308, 0.1, 4, 4), (0.0, 0.0, 0.1, 0.1, -1, 4)):
        with pytest.raises(R.RbfError) as e:
            R.rbf_evaluate_lattice(h, *bad)
        assert e.value.status == R.RBF_EINVAL, bad
    assert R.rbf_evaluate_lattice(h, 0.0, 0.0, 0.1, 0.1, 0, 5).shape == (5, 0)
    # before any solve
    h2 = R.rbf_setup(pts, w.values(pts), w.sigma, w.cutoff, 1)
    try:
        with pytest.raises(R.RbfError) as e:
            R.rbf_evaluate_lattice(h2, 0.0, 0.0, 0.1, 0.1, 4, 4)
        assert e.value.status == R.RBF_ESTATE
    finally:
        R.rbf_destroy(h2)


def test_lattice_box_truncated_equals_box_evaluation(torch_dev, oracle_mod):
    w = W.MINI
    pts = w.points()
    s = w.sigma
    h = R.rbf_setup(pts, w.values(pts), s, w.cutoff, 1)
    try:
        R.rbf_set_geometry(h, 5 * s, 9.5 * s, 17 * s)
        R.rbf_solve(h, pts.shape[0], R.default_opts(rtol=1e-10))
        x0, y0, hx, hy, nx, ny = -1.1, -0.95, 0.7 * w.h, 0.9 * w.h, 70, 50
        tg = lattice(x0, y0, hx, hy, nx, ny)
        assert np.array_equal(R.rbf_evaluate_lattice(h, x0, y0, hx, hy, nx, ny).ravel(),
                              R.rbf_evaluate(h, tg))
    finally:
        R.rbf_destroy(h)


def test_lattice_is_deterministic(torch_dev, solved):
    h, P, pts, lam, w = solved
    args = lattices(w)["fine_wide"]
    assert np.array_equal(R.rbf_evaluate_lattice(h, *args), R.rbf_evaluate_lattice(h, *args))
