"""Edge cases of the GPU path, through the C ABI (-m gpu).

Degenerate problems against closed forms: one point (lambda = f / phi(0)),
two points (the 2x2 system), one cell holding every point (the restricted
additive Schwarz preconditioner is then the exact inverse, so right-
preconditioned GMRES stops after one iteration, Section 2.2).  A point set
with empty cells (an annulus: cells with no own points build no block and
own no rows), and the largest local blocks the workloads here reach (local
blocks of up to 1444 points, n_p = 1472: 23 block columns of the
factorisation; up to 169 points per cell: three passes of 64 right-hand
sides in the centre-row solves), each against the oracle.  A cell holding
more targets than one workgroup of the list matvec serves (its targets split
over two groups staging the same neighbourhood), against the oracle.  A local
block above RBF_MAX_BLOCK is refused with RBF_ELIMIT.
"""
import sys

import numpy as np
import pytest

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


def lattice(n, h_over_sigma, seed, jitter=0.1):
    rng = np.random.default_rng(seed)
    h = 2.0 / n
    xs = -1 + (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(xs, xs)
    pts = np.stack([X.ravel(), Y.ravel()], 1) + rng.uniform(-jitter * h, jitter * h, (n * n, 2))
    return pts, h / h_over_sigma


def annulus():
    pts, sigma = lattice(40, 0.9, 21)
    r = np.hypot(pts[:, 0], pts[:, 1])
    return pts[(r > 0.55) & (r < 1.0)], sigma, 6 * sigma


def largest_blocks():
    pts, sigma = lattice(60, 0.95, 22)
    return pts, sigma, 12 * sigma


def gpu_matvec(torch, h, w):
    dw = torch.tensor(w, device="cuda", dtype=torch.float64)
    dy = torch.empty_like(dw)
    R.rbf_matvec_device(h, dw, dy, R.RBF_FP64, R.RBF_ORDER_ORIGINAL, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return dy.cpu().numpy()


def gpu_rasm(torch, h, v):
    dv = torch.tensor(v, device="cuda", dtype=torch.float64)
    dz = torch.empty_like(dv)
    R.rbf_precond_apply_device(h, dv, dz, R.RBF_FP64, R.RBF_ORDER_ORIGINAL,
                               torch.cuda.current_stream())
    torch.cuda.synchronize()
    return dz.cpu().numpy()


def test_single_point(torch_dev):
    say("one point")
    sigma, f = 0.1, np.array([2.0])
    h = R.rbf_setup(np.array([[0.3, -0.2]]), f, sigma, 6 * sigma, 1)
    try:
        for prec, rtol in ((R.RBF_FP64, 1e-14), (R.RBF_MIXED, 1e-12)):
            lam, info, st = R.rbf_solve(h, 1, R.default_opts(rtol=rtol, precision=prec))
            assert st == R.RBF_OK
            # A = [phi(0)] = [1 / (2 pi sigma^2)]
            assert abs(lam[0] - f[0] * 2 * np.pi * sigma * sigma) <= rtol * abs(lam[0])
    finally:
        R.rbf_destroy(h)


def test_two_points(torch_dev):
    say("two points")
    sigma = 0.1
    pts = np.array([[0.0, 0.0], [0.05, 0.02]])
    f = np.array([1.0, -0.5])
    h = R.rbf_setup(pts, f, sigma, 6 * sigma, 1)
    try:
        lam, info, st = R.rbf_solve(h, 2, R.default_opts(rtol=1e-14))
    finally:
        R.rbf_destroy(h)
    d2 = float(np.sum((pts[0] - pts[1]) ** 2))
    e = np.exp(-d2 / (2 * sigma * sigma))
    A = np.array([[1.0, e], [e, 1.0]]) / (2 * np.pi * sigma * sigma)
    ref = np.linalg.solve(A, f)
    assert np.linalg.norm(lam - ref) <= 1e-13 * np.linalg.norm(ref), (lam, ref)
    assert info.iterations == 1


def test_single_subdomain(torch_dev, oracle_mod):
    """Every point in one cell: M^-1 = A^-1, so one GMRES iteration reaches
    cond(A) u, far below the tolerance on a jittered lattice at h/sigma = 1."""
    say("one cell")
    rng = np.random.default_rng(3)
    sigma = 0.02
    xs = (np.arange(12) - 5.5) * sigma
    X, Y = np.meshgrid(xs, xs)
    pts = np.stack([X.ravel(), Y.ravel()], 1) + rng.uniform(-0.1 * sigma, 0.1 * sigma, (144, 2))
    f = W.gaussian_vortex(pts)
    h = R.rbf_setup(pts, f, sigma, 60 * sigma, 1)
    try:
        _, (ncx, ncy) = R.rbf_grid(h)
        assert (ncx, ncy) == (1, 1)
        lam, info, st = R.rbf_solve(h, pts.shape[0], R.default_opts(rtol=1e-12))
    finally:
        R.rbf_destroy(h)
    assert info.iterations == 1
    P = oracle_mod.Problem(pts, sigma, 60 * sigma, 1)
    try:
        assert P.rel_residual(f, lam) <= residual_gate(P, f, lam, 1e-12)
    finally:
        P.close()


def test_empty_cells(torch_dev, oracle_mod):
    """An annulus: the cells inside the hole have no points."""
    pts, sigma, cutoff = annulus()
    say("annulus", pts.shape[0])
    f = W.gaussian_vortex(pts)
    h = R.rbf_setup(pts, f, sigma, cutoff, 1)
    P = oracle_mod.Problem(pts, sigma, cutoff, 1)
    try:
        _, (ncx, ncy) = R.rbf_grid(h)
        cell_of, perm, cs = R.rbf_binning(h, pts.shape[0])
        o_cell, o_perm, o_cs = P.binning()
        assert np.array_equal(cell_of, o_cell) and np.array_equal(perm, o_perm)
        assert np.array_equal(cs.astype(np.int64), o_cs)
        assert int(np.sum(np.diff(o_cs) == 0)) >= 1, "the annulus has empty cells"
        w = W.random_weights(pts.shape[0], 31)
        y = gpu_matvec(torch_dev, h, w)
        assert np.max(np.abs(y - P.matvec(w)) / P.matvec(np.abs(w))) <= 1e-13
        P.rasm_setup()
        z = gpu_rasm(torch_dev, h, w)
        zo = P.rasm_apply(w)
        assert np.linalg.norm(z - zo) <= 1e-7 * np.linalg.norm(zo)
        lam, info, st = R.rbf_solve(h, pts.shape[0], R.default_opts(rtol=1e-12))
        assert P.rel_residual(f, lam) <= residual_gate(P, f, lam, 1e-12)
        _, oinfo = P.gmres(f, 30, 1e-12)
        assert abs(info.iterations - oinfo.iterations) <= 2
    finally:
        R.rbf_destroy(h)
        P.close()


def test_largest_blocks(torch_dev, oracle_mod):
    """Local blocks of up to 1444 points (n_p = 1472) and cells of up to 169
    points: the centre rows of the largest block are backward-stable rows of
    its inverse, the RASM apply and the FP64 and mixed solves match the
    oracle."""
    pts, sigma, cutoff = largest_blocks()
    say("largest blocks", pts.shape[0])
    from tests import bruteforce as bf
    f = W.gaussian_vortex(pts)
    h = R.rbf_setup(pts, f, sigma, cutoff, 1)
    P = oracle_mod.Problem(pts, sigma, cutoff, 1)
    try:
        _, (ncx, ncy) = R.rbf_grid(h)
        _, _, o_cs = P.binning()
        own = np.diff(o_cs)
        sizes = []
        for cell in range(ncx * ncy):
            mem, _, _ = P.rasm_block(cell, with_factor=False)
            sizes.append(len(mem))
        big = int(np.argmax(sizes))
        assert sizes[big] > 1400 and own.max() > 128, (sizes[big], own.max())
        u = np.finfo(float).eps / 2
        for cell in (big, int(np.argmax(own))):
            mem, Z = R.rbf_precond_block(h, cell, R.RBF_FP64)
            o_mem, kc, _ = P.rasm_block(cell, with_factor=False)
            assert np.array_equal(mem, o_mem)
            A = bf.dense_matrix(pts[mem], sigma, None)
            n = len(mem)
            E = np.eye(n)[n - kc:]
            res = np.linalg.norm(Z @ A - E, 2)
            bound = 10 * n * u * np.linalg.norm(Z, 2) * np.linalg.norm(A, 2)
            say("largest block", cell, n, kc, res / bound)
            assert res <= bound, (cell, res, bound)
        P.rasm_setup()
        v = W.random_weights(pts.shape[0], 41)
        z = gpu_rasm(torch_dev, h, v)
        zo = P.rasm_apply(v)
        assert np.linalg.norm(z - zo) <= 1e-7 * np.linalg.norm(zo)
        lam, info, st = R.rbf_solve(h, pts.shape[0], R.default_opts(rtol=1e-12))
        assert P.rel_residual(f, lam) <= residual_gate(P, f, lam, 1e-12)
        _, oinfo = P.gmres(f, 30, 1e-12)
        assert abs(info.iterations - oinfo.iterations) <= 2
        lam32, info32, st32 = R.rbf_solve(h, pts.shape[0],
                                          R.default_opts(rtol=1e-12, precision=R.RBF_MIXED))
        assert st32 == R.RBF_OK
        assert P.rel_residual(f, lam32) <= residual_gate(P, f, lam32, 1e-12)
    finally:
        R.rbf_destroy(h)
        P.close()


def test_block_limit(torch_dev):
    """A local block above RBF_MAX_BLOCK points is refused, not truncated."""
    pts, sigma = lattice(50, 0.9, 23)
    say("block limit", pts.shape[0])
    f = W.gaussian_vortex(pts)
    h = R.rbf_setup(pts, f, sigma, 13 * sigma, 1)
    try:
        with pytest.raises(R.RbfError) as e:
            R.rbf_solve(h, pts.shape[0], R.default_opts(rtol=1e-10))
        assert e.value.status == R.RBF_ELIMIT
    finally:
        R.rbf_destroy(h)


def crowded_cell():
    """A jittered 30x30 lattice (h/sigma = 0.8, cutoff 6 sigma: a 4x4 grid of
    cells of ~56 points) plus 700 points drawn uniformly in a disk of radius
    2 sigma at the centre of cell (1, 1): that cell holds ~756 targets, more
    than one workgroup of the list matvec serves (8 units of 64), so its
    targets are split over two groups that stage the same neighbourhood."""
    pts, sigma = lattice(30, 0.8, 31)
    cutoff = 6 * sigma
    rng = np.random.default_rng(32)
    x0, y0 = pts[:, 0].min(), pts[:, 1].min()
    c = np.array([x0 + 1.5 * cutoff, y0 + 1.5 * cutoff])
    r = 2 * sigma * np.sqrt(rng.uniform(0, 1, 700))
    t = rng.uniform(0, 2 * np.pi, 700)
    extra = c + np.stack([r * np.cos(t), r * np.sin(t)], 1)
    return np.concatenate([pts, extra]), sigma, cutoff


def test_cell_split_over_groups(torch_dev, oracle_mod):
    torch = torch_dev
    pts, sigma, cutoff = crowded_cell()
    n = pts.shape[0]
    say("crowded cell", n)
    h = R.rbf_setup(pts, np.ones(n), sigma, cutoff, 1)
    try:
        P = oracle_mod.Problem(pts, sigma, cutoff, 1)
        cell_of, _, cs = R.rbf_binning(h, n)
        assert np.max(np.diff(cs)) > 512
        nnb, _ = R.rbf_neighbor_counts(h, n)
        _, o_nnb = P.matvec(np.ones(n), with_counts=True)
        assert np.array_equal(nnb, o_nnb)
        w = np.random.default_rng(33).uniform(-1, 1, n)
        yo = P.matvec(w)
        scale = P.matvec(np.abs(w))
        y = gpu_matvec(torch, h, w)
        assert np.max(np.abs(y - yo) / scale) <= 1e-13
        dw = torch.tensor(w, device="cuda", dtype=torch.float64)
        dy = torch.empty_like(dw)
        R.rbf_matvec_device(h, dw, dy, R.RBF_MIXED, R.RBF_ORDER_ORIGINAL,
                            torch.cuda.current_stream())
        torch.cuda.synchronize()
        assert np.max(np.abs(dy.cpu().numpy() - yo) / scale) <= 2e-5
    finally:
        R.rbf_destroy(h)


def test_nan_residual_reported(torch_dev, oracle_mod):
    """Finite data whose norm overflows (f = 1e200 everywhere): the residual
    norm is Inf / Inf, reported as RBF_ENAN by both forms and by the oracle."""
    w = W.MINI
    pts = w.points()
    f = np.full(w.n, 1e200)
    say("enan", w.n)
    h = R.rbf_setup(pts, f, w.sigma, w.cutoff, 1)
    try:
        for prec in (R.RBF_FP64, R.RBF_MIXED):
            _, info, st = R.rbf_solve(h, w.n, R.default_opts(rtol=1e-10, precision=prec),
                                      ok=(R.RBF_ENAN,))
            assert st == R.RBF_ENAN
    finally:
        R.rbf_destroy(h)
    P = oracle_mod.Problem(pts, w.sigma, w.cutoff, 1)
    _, oinfo = P.gmres(f, 30, 1e-10, raise_on_error=False)
    assert oinfo.status == 8          # ORC_ENAN


def test_not_positive_definite_reported(torch_dev, oracle_mod):
    """h/sigma = 0.1 and a cutoff wider than the point set: one local block of
    all 900 points whose Gaussian matrix is SPD in exact arithmetic but of
    numerical rank far below 900 (its condition number is about
    exp(pi^2 sigma^2 / h^2), e^987), so a Cholesky pivot comes out <= 0 in
    FP64: RBF_ENOTPD from the GPU factorisation and ENOTPD from the oracle's."""
    rng = np.random.default_rng(71)
    n = 30
    hh = 2.0 / n
    xs = -1 + (np.arange(n) + 0.5) * hh
    X, Y = np.meshgrid(xs, xs)
    pts = np.stack([X.ravel(), Y.ravel()], 1) + rng.uniform(-0.1 * hh, 0.1 * hh, (n * n, 2))
    sigma = hh / 0.1
    cutoff = 6 * sigma
    f = W.gaussian_vortex(pts)
    say("enotpd", pts.shape[0])
    h = R.rbf_setup(pts, f, sigma, cutoff, 1)
    try:
        assert R.rbf_grid(h)[1] == (1, 1)
        with pytest.raises(R.RbfError) as e:
            R.rbf_precond_setup(h, R.RBF_FP64)
        assert e.value.status == R.RBF_ENOTPD
        with pytest.raises(R.RbfError) as e:
            R.rbf_solve(h, pts.shape[0], R.default_opts(rtol=1e-10))
        assert e.value.status == R.RBF_ENOTPD
    finally:
        R.rbf_destroy(h)
    P = oracle_mod.Problem(pts, sigma, cutoff, 1)
    with pytest.raises(oracle_mod.OracleError) as e:
        P.rasm_setup()
    assert e.value.code == 5          # ORC_ENOTPD


def test_breakdown_is_reported_consistently(torch_dev):
    """One point: the preconditioned operator is a scalar, so the first Arnoldi
    step leaves nothing after orthogonalisation (an exact breakdown).  With
    rtol = 0 the solve then ends after that step: RBF_OK if the true residual
    is exactly zero, RBF_EBREAKDOWN (with the residual reported) otherwise."""
    sigma, f = 0.1, np.array([2.0])
    h = R.rbf_setup(np.array([[0.3, -0.2]]), f, sigma, 6 * sigma, 1)
    try:
        lam, info, st = R.rbf_solve(h, 1, R.default_opts(rtol=0.0),
                                    ok=(R.RBF_OK, R.RBF_EBREAKDOWN))
    finally:
        R.rbf_destroy(h)
    say("breakdown", R.status_name(st), info.rel_residual, info.iterations)
    assert info.iterations == 1 and info.restarts == 1
    assert (st == R.RBF_EBREAKDOWN) == (info.rel_residual > 0.0)
    assert abs(lam[0] - f[0] * 2 * np.pi * sigma * sigma) <= 4e-16 * abs(lam[0])


def test_resume_from_lambda0(torch_dev, oracle_mod):
    """Checkpoint and resume: a solve to 1e-6 whose weights seed a second
    solve to 1e-12 reaches the same bar as a fresh solve, in fewer
    iterations than the fresh one; the set-up time of the handle is
    reported."""
    w = W.C0
    pts = w.points()
    f = w.values(pts)
    say("resume", w.n)
    h = R.rbf_setup(pts, f, w.sigma, w.cutoff, 1)
    try:
        # the history pointer is valid until the next call on the handle:
        # copy each info out at once
        lam1, i1, _ = R.rbf_solve(h, w.n, R.default_opts(rtol=1e-6))
        i1 = i1.as_dict()
        lam2, i2, _ = R.rbf_solve(h, w.n, R.default_opts(rtol=1e-12), lambda0=lam1)
        i2 = i2.as_dict()
        lam3, i3, _ = R.rbf_solve(h, w.n, R.default_opts(rtol=1e-12))
        i3 = i3.as_dict()
    finally:
        R.rbf_destroy(h)
    say("resume iterations", i1["iterations"], i2["iterations"], i3["iterations"])
    assert i1["rel_residual"] <= 1e-6 and i2["rel_residual"] <= 1e-12
    # the resumed solve starts where the first one stopped
    assert i2["history"][0] == pytest.approx(i1["rel_residual"], rel=1e-6)
    assert i2["iterations"] < i3["iterations"]
    assert i1["t_init"] > 0 and i1["t_init"] == i2["t_init"] == i3["t_init"]
    assert i2["t_pcsetup"] < i1["t_pcsetup"] and i3["t_pcsetup"] < i1["t_pcsetup"]
    P = oracle_mod.Problem(pts, w.sigma, w.cutoff, 1)
    assert P.rel_residual(f, lam2) <= residual_gate(P, f, lam2, 1e-12)


def test_mixed_refinement_never_returns_a_worse_iterate(torch_dev, oracle_mod):
    """h/sigma = 0.6 (kappa(A) u32 >> 1): FP32 inner solves cannot reduce the
    FP64 residual for long.  An outer step that does not lower it is undone
    and the solve stops with RBF_ENOCONV: the reported residual is the
    smallest of the history (each accepted step lowered it), it is below the
    starting one, and the oracle's residual of the returned weights agrees
    with it, so the returned iterate is the one the residual belongs to."""
    pts, sigma = lattice(60, 0.6, 31)
    f = W.gaussian_vortex(pts, 0.2)
    n = pts.shape[0]
    say("mixed refinement at h/sigma 0.6", n)
    h = R.rbf_setup(pts, f, sigma, 6 * sigma, 1)
    try:
        lam, info, st = R.rbf_solve(h, n, R.default_opts(rtol=1e-12, precision=R.RBF_MIXED,
                                                          max_iters=900),
                                    ok=(R.RBF_ENOCONV,))
        d = info.as_dict()
    finally:
        R.rbf_destroy(h)
    hist = d["history"]
    say("outer", d["outer_iterations"], "iterations", d["iterations"], "history", hist)
    assert st == R.RBF_ENOCONV
    assert np.all(np.isfinite(lam))
    assert d["rel_residual"] == min(hist)
    assert d["rel_residual"] < hist[0]
    assert all(b < a for a, b in zip(hist[:-2], hist[1:-1]))   # accepted steps
    P = oracle_mod.Problem(pts, sigma, 6 * sigma, 1)
    res = P.rel_residual(f, lam)
    slack = residual_gate(P, f, lam, 0.0)
    say("oracle residual", res, "reported", d["rel_residual"], "slack", slack)
    assert abs(res - d["rel_residual"]) <= slack


def test_library_before_torch_load_order(torch_dev):
    """A process that loads the library before it initialises PyTorch's device
    still finds the GPU (the binding brings PyTorch's HIP runtime in first):
    a small solve in a child process, in that order."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import paper_0909_5413_amd as R; from paper_0909_5413_amd import workloads as W; "
            "R.lib(); import torch; torch.cuda.init(); w = W.MINI; p = w.points(); "
            "h = R.rbf_setup(p, w.values(p), w.sigma, w.cutoff, 1); "
            "lam, info, st = R.rbf_solve(h, w.n, R.default_opts(rtol=1e-10)); "
            "s = R.rbf_server_create(); R.rbf_server_destroy(s); R.rbf_destroy(h); "
            "print('ok', st, info.iterations)")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=180)
    say("child", r.returncode, r.stdout.strip(), r.stderr.strip()[-300:])
    assert r.returncode == 0 and r.stdout.startswith("ok 0"), r.stderr[-2000:]
